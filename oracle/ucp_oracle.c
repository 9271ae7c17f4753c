/*
 * Plain FP64 CPU oracle for the marginal-cost solver on Witsenhausen's
 * counterexample, and (at the end of this file) on the zero-delay
 * source-channel coding problem and the two-dimensional counterexample.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously correct statement
 * of what the GPU path computes.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark load it; the product path never does.
 * It shares no code, header or constant with the HIP library.
 *
 * Problem (Section V-A): x0 ~ prior f, y0 = x0, x1 = x0 + u0(y0),
 * y1 = x1 + w with w ~ N(0,1), x2 = x1 - u1(y1),
 * J = E[k^2 u0(y0)^2 + x2^2].
 *
 * Discretisation (Section III-D, "Initialization"): each controller is a
 * step function on a linearly spaced grid over [a,b]; every integral is
 * taken by the rectangle rule with weight (b-a)/(d-1) at each node.
 *
 * Arithmetic: IEEE FP64, exp() from libm, every sum in ascending index
 * order, dense over all grid nodes (no window), no fast-math and no FMA
 * contraction.  OpenMP splits only the independent outer index (Section
 * IV-A: the points of one controller are independent), so results do not
 * depend on the thread count.
 *
 * Parity status of each function is stated in its comment; every function
 * here is pinned by the CPU tests against closed forms, exact discrete
 * identities or a high-precision brute force.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_COMP 8
#define ORC_TAU64 1e-12 /* relative tie band of the selection rule, unless the search sets one */

/* Problem description: stage-1 weight k, a Gaussian-mixture prior for x0
 * (one component = the paper's N(0, sigma^2)), the two grids, and the
 * standard deviation of the Gaussian noise w (Section V-A fixes 1; 0 also
 * selects 1).  The coding and two-dimensional problems below have noises
 * of their own and ignore noise_sd. */
typedef struct {
  double k;
  int32_t n_comp;
  int32_t pad_;
  double w[ORC_MAX_COMP];
  double mu[ORC_MAX_COMP];
  double sd[ORC_MAX_COMP];
  double x_lo, x_hi;
  int64_t n_x;
  double y_lo, y_hi;
  int64_t n_y;
  double noise_sd;
} orc_problem;

static double orc_noise_sd(const orc_problem* p) { return p->noise_sd > 0.0 ? p->noise_sd : 1.0; }

/* Coarse-to-fine search settings for the u0 update.  tie_rel64 is the
 * relative tie band of the selection rule (0 selects ORC_TAU64);
 * band_rel32 belongs to the FP32 pre-selection of the GPU path and has no
 * meaning here (the layout matches the library's search record). */
typedef struct {
  double u_lo, u_hi;
  int32_t levels;
  int32_t cands;
  double tie_rel64;
  double band_rel32;
} orc_search;

static double orc_tau(const orc_search* s) { return s->tie_rel64 > 0.0 ? s->tie_rel64 : ORC_TAU64; }

static const double ORC_PI = 3.14159265358979323846264338327950288;

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Grid node i of a linspace over [lo,hi] with n nodes (Section III-D). */
static double orc_node(double lo, double hi, int64_t n, int64_t i) {
  double step = (hi - lo) / (double)(n - 1);
  return lo + (double)i * step;
}

void orc_grid(double lo, double hi, int64_t n, double* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = orc_node(lo, hi, n, i);
}

/* Prior density of x0 and its logarithm at every x-grid node.
 * Section V-A fixes x0 ~ N(0, sigma^2); a mixture generalises it.
 * log f is a log-sum-exp over components so it never takes log(0). */
void orc_prior(const orc_problem* p, double* f, double* logf) {
  for (int64_t i = 0; i < p->n_x; ++i) {
    double x = orc_node(p->x_lo, p->x_hi, p->n_x, i);
    double lc[ORC_MAX_COMP];
    double sum = 0.0;
    double lmax = -INFINITY;
    for (int c = 0; c < p->n_comp; ++c) {
      double d = (x - p->mu[c]) / p->sd[c];
      double dens = p->w[c] * exp(-0.5 * d * d) / (p->sd[c] * sqrt(2.0 * ORC_PI));
      sum += dens;
      lc[c] = log(p->w[c]) - log(p->sd[c]) - 0.5 * log(2.0 * ORC_PI) - 0.5 * d * d;
      if (lc[c] > lmax) lmax = lc[c];
    }
    double acc = 0.0;
    for (int c = 0; c < p->n_comp; ++c) acc += exp(lc[c] - lmax);
    if (f) f[i] = sum;
    if (logf) logf[i] = lmax + log(acc);
  }
}

/* Noise density phi(t) of w ~ N(0,1) (Section V-A). */
static double orc_phi(double t) { return exp(-0.5 * t * t) / sqrt(2.0 * ORC_PI); }

/* Density of w ~ N(0, s^2). */
static double orc_phi_s(double t, double s) {
  double u = t / s;
  return exp(-0.5 * u * u) / (s * sqrt(2.0 * ORC_PI));
}

/* B(u; x) = L_0(u, x) / f(x): the marginal cost of the first controller
 * at the point x0 = x with u0(x) = u, divided by the prior density.
 * Marginal cost C_0 (Section III-A, definition of C_m) applied to the
 * Witsenhausen objective: k^2 u^2 + integral over y of
 * phi(y - x - u) (x + u - u1(y))^2, by the rectangle rule on the y grid. */
double orc_B(const orc_problem* p, const double* u1, double x, double u) {
  double dy = (p->y_hi - p->y_lo) / (double)(p->n_y - 1);
  double sw = orc_noise_sd(p);
  double z = x + u;
  double s = 0.0;
  for (int64_t j = 0; j < p->n_y; ++j) {
    double y = orc_node(p->y_lo, p->y_hi, p->n_y, j);
    double e = z - u1[j];
    s += orc_phi_s(y - z, sw) * e * e;
  }
  return p->k * p->k * u * u + dy * s;
}

/* L_0(u; x_i) = f_i * B(u; x_i) for a set of candidates per point.
 * u and out are row-major [n_x][n_cand]. */
void orc_marginal_cost(const orc_problem* p, const double* u1, const double* u,
                       int64_t n_cand, double* out) {
  double* f = (double*)malloc(sizeof(double) * (size_t)p->n_x);
  orc_prior(p, f, NULL);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < p->n_x; ++i) {
    double x = orc_node(p->x_lo, p->x_hi, p->n_x, i);
    for (int64_t c = 0; c < n_cand; ++c)
      out[i * n_cand + c] = f[i] * orc_B(p, u1, x, u[i * n_cand + c]);
  }
  free(f);
}

/* Selection among a finite candidate set (the improvement rule of
 * Section III-B on a finite set): the members whose B lies within a
 * relative band tau of the minimum are ties; among them the one nearest
 * the incumbent u_inc wins, and an equal distance goes to the smaller u.
 * Returns the index of the chosen member. */
static int orc_select(int n, const double* c, const double* B, double u_inc, double tau) {
  double m = B[0];
  for (int s = 1; s < n; ++s)
    if (B[s] < m) m = B[s];
  double thr = m * (1.0 + tau);
  int best = -1;
  double bd = 0.0;
  for (int s = 0; s < n; ++s) {
    if (!(B[s] <= thr)) continue;
    double d = fabs(c[s] - u_inc);
    if (best < 0 || d < bd || (d == bd && c[s] < c[best])) {
      best = s;
      bd = d;
    }
  }
  return best;
}

/* Spacing of the candidate grid at every level of the coarse-to-fine
 * search: level 0 spans [u_lo,u_hi] with K nodes; each later level spans
 * the neighbour bracket [c* - h_prev, c* + h_prev] with K nodes. */
void orc_spacings(const orc_search* s, double* h) {
  h[0] = (s->u_hi - s->u_lo) / (double)(s->cands - 1);
  for (int l = 1; l < s->levels; ++l) h[l] = 2.0 * h[l - 1] / (double)(s->cands - 1);
}

static double orc_clamp(double v, double lo, double hi) {
  if (v < lo) return lo;
  if (v > hi) return hi;
  return v;
}

/* Pointwise improvement of u0 at one point (Corollary 1 and the update
 * rule of Section III-B): a coarse-to-fine search of argmin_u B(u; x_i),
 * the best-so-far carried from level to level, and the incumbent u0_i
 * kept in the final comparison so the update never raises the cost. */
double orc_cd_B(const orc_problem* p, double lam, const double* u1, double x, double u);

/* B of the problem being searched: model 0 is the Witsenhausen objective
 * above, model 1 the source-channel coding objective further below (with
 * stage-0 weight lam). */
static double orc_model_B(int model, double lam, const orc_problem* p, const double* u1, double x,
                          double u) {
  return model == 1 ? orc_cd_B(p, lam, u1, x, u) : orc_B(p, u1, x, u);
}

/* visit (NULL, or levels * cands + 1 entries) receives every position whose
 * B was evaluated, level by level, the incumbent last: the work count of the
 * CPU baseline. */
static double orc_argmin_point(const orc_problem* p, const orc_search* s,
                               const double* u1, const double* h, int64_t i,
                               double u_inc, double* B_out, int model, double lam, double* visit) {
  int K = s->cands;
  double x = orc_node(p->x_lo, p->x_hi, p->n_x, i);
  double* c = (double*)malloc(sizeof(double) * (size_t)(K + 1));
  double* B = (double*)malloc(sizeof(double) * (size_t)(K + 1));
  /* level 0: the global grid over [u_lo, u_hi] */
  for (int q = 0; q < K; ++q) {
    c[q] = s->u_lo + (double)q * h[0];
    B[q] = orc_model_B(model, lam, p, u1, x, c[q]);
    if (visit) visit[q] = c[q];
  }
  const double tau = orc_tau(s);
  int b = orc_select(K, c, B, u_inc, tau);
  double cs = c[b], Bs = B[b];
  /* finer levels around the best so far, which stays in the set */
  for (int l = 1; l < s->levels; ++l) {
    for (int q = 0; q < K; ++q) {
      c[q] = orc_clamp(cs - h[l - 1] + (double)q * h[l], s->u_lo, s->u_hi);
      B[q] = orc_model_B(model, lam, p, u1, x, c[q]);
      if (visit) visit[l * K + q] = c[q];
    }
    c[K] = cs;
    B[K] = Bs;
    b = orc_select(K + 1, c, B, u_inc, tau);
    cs = c[b];
    Bs = B[b];
  }
  /* acceptance against the incumbent */
  c[0] = cs;
  B[0] = Bs;
  c[1] = u_inc;
  B[1] = orc_model_B(model, lam, p, u1, x, u_inc);
  if (visit) visit[s->levels * K] = u_inc;
  b = orc_select(2, c, B, u_inc, tau);
  double r = c[b];
  if (B_out) *B_out = B[b];
  free(c);
  free(B);
  return r;
}

/* One u0 update over the listed points (rows == NULL: every point) of
 * model 0 or 1 (see orc_model_B).  u0_out[r] and B_out[r] are indexed like
 * rows. */
static void orc_argmin_model(const orc_problem* p, const orc_search* s, const double* u1,
                             const double* u0_in, const int64_t* rows, int64_t n_rows,
                             double* u0_out, double* B_out, int model, double lam, double* visits) {
  double h[64];
  orc_spacings(s, h);
  int64_t n = rows ? n_rows : p->n_x;
  const int64_t nv = (int64_t)s->levels * s->cands + 1;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < n; ++r) {
    int64_t i = rows ? rows[r] : r;
    double Bv;
    u0_out[r] = orc_argmin_point(p, s, u1, h, i, u0_in[i], &Bv, model, lam, visits ? visits + r * nv : NULL);
    if (B_out) B_out[r] = Bv;
  }
}

/* orc_argmin that also reports the positions evaluated per listed row
 * (visits: [n_rows][levels * cands + 1]). */
void orc_argmin_visits(const orc_problem* p, const orc_search* s, const double* u1,
                       const double* u0_in, const int64_t* rows, int64_t n_rows,
                       double* u0_out, double* visits) {
  orc_argmin_model(p, s, u1, u0_in, rows, n_rows, u0_out, NULL, 0, 0.0, visits);
}

/* Thread count of the OpenMP loops (n < 1: the runtime's default). */
void orc_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
  (void)n;
#endif
}

void orc_argmin(const orc_problem* p, const orc_search* s, const double* u1,
                const double* u0_in, const int64_t* rows, int64_t n_rows,
                double* u0_out, double* B_out) {
  orc_argmin_model(p, s, u1, u0_in, rows, n_rows, u0_out, B_out, 0, 0.0, NULL);
}

/* Second controller by its closed form: u1(y) = E[x1 | y1 = y], the exact
 * minimiser of the discrete marginal cost C_1(v, y) (the closed form the
 * paper credits to the earlier algorithm, Section IV-B).  With
 * l_ij = log f_i - (y_j - x1_i)^2 / 2 and M_j = max_i l_ij,
 * u1_j = sum_i x1_i e^(l_ij - M_j) / sum_i e^(l_ij - M_j).
 * rows == NULL: every y node; else only the listed nodes (out indexed
 * like rows). */
void orc_update_u1(const orc_problem* p, const double* u0, const int64_t* rows,
                   int64_t n_rows, double* u1_out) {
  double* logf = (double*)malloc(sizeof(double) * (size_t)p->n_x);
  double* x1 = (double*)malloc(sizeof(double) * (size_t)p->n_x);
  orc_prior(p, NULL, logf);
  for (int64_t i = 0; i < p->n_x; ++i) x1[i] = orc_node(p->x_lo, p->x_hi, p->n_x, i) + u0[i];
  const double sw = orc_noise_sd(p);
  int64_t n = rows ? n_rows : p->n_y;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < n; ++r) {
    int64_t j = rows ? rows[r] : r;
    double y = orc_node(p->y_lo, p->y_hi, p->n_y, j);
    double M = -INFINITY;
    for (int64_t i = 0; i < p->n_x; ++i) {
      double d = (y - x1[i]) / sw;
      double l = logf[i] - 0.5 * d * d;
      if (l > M) M = l;
    }
    double num = 0.0, den = 0.0;
    for (int64_t i = 0; i < p->n_x; ++i) {
      double d = (y - x1[i]) / sw;
      double e = exp(logf[i] - 0.5 * d * d - M);
      num += x1[i] * e;
      den += e;
    }
    u1_out[r] = num / den;
  }
  free(logf);
  free(x1);
}

/* Objective J[U] of Section V-A by the rectangle rule in x0 and y:
 * J = dx * sum_i f_i [k^2 u0_i^2 + dy * sum_j phi(y_j - x1_i)(x1_i - u1_j)^2]. */
double orc_objective(const orc_problem* p, const double* u0, const double* u1) {
  double dx = (p->x_hi - p->x_lo) / (double)(p->n_x - 1);
  double dy = (p->y_hi - p->y_lo) / (double)(p->n_y - 1);
  const double sw = orc_noise_sd(p);
  double* f = (double*)malloc(sizeof(double) * (size_t)p->n_x);
  double* row = (double*)malloc(sizeof(double) * (size_t)p->n_x);
  orc_prior(p, f, NULL);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < p->n_x; ++i) {
    double x1 = orc_node(p->x_lo, p->x_hi, p->n_x, i) + u0[i];
    double s = 0.0;
    for (int64_t j = 0; j < p->n_y; ++j) {
      double y = orc_node(p->y_lo, p->y_hi, p->n_y, j);
      double e = x1 - u1[j];
      s += orc_phi_s(y - x1, sw) * e * e;
    }
    row[i] = f[i] * (p->k * p->k * u0[i] * u0[i] + dy * s);
  }
  double J = 0.0;
  for (int64_t i = 0; i < p->n_x; ++i) J += row[i];
  free(f);
  free(row);
  return dx * J;
}

/* The solve loop: u1 from the initial u0, then `iters` rounds of
 * (u0 update, u1 update), J recorded after each round.  This is the
 * controller loop of Algorithm 1 with M = 2 controllers visited in order,
 * the u0 update done by the coarse-to-fine search and the u1 update by its
 * closed form.  J_hist has iters + 1 entries. */
void orc_solve(const orc_problem* p, const orc_search* s, int32_t iters,
               const double* u0_init, double* u0_out, double* u1_out, double* J_hist) {
  double* u0 = (double*)malloc(sizeof(double) * (size_t)p->n_x);
  double* nxt = (double*)malloc(sizeof(double) * (size_t)p->n_x);
  memcpy(u0, u0_init, sizeof(double) * (size_t)p->n_x);
  orc_update_u1(p, u0, NULL, 0, u1_out);
  J_hist[0] = orc_objective(p, u0, u1_out);
  for (int32_t t = 1; t <= iters; ++t) {
    orc_argmin(p, s, u1_out, u0, NULL, 0, nxt, NULL);
    memcpy(u0, nxt, sizeof(double) * (size_t)p->n_x);
    orc_update_u1(p, u0, NULL, 0, u1_out);
    J_hist[t] = orc_objective(p, u0, u1_out);
  }
  memcpy(u0_out, u0, sizeof(double) * (size_t)p->n_x);
  free(u0);
  free(nxt);
}

/* ------------------------------------------------------------------------
 * Zero-delay source-channel coding (Section V-B): x0 ~ prior f (the
 * paper's N(0,1), or a mixture), y0 = x0, x1 = u0(y0) + w with
 * w ~ U(-1, 1), y1 = x1, J = E[lam u0(y0)^2 + (u1(y1) - x0)^2].
 * The same grids and rectangle rule as above; p->k is not used, the stage-0
 * weight is lam.  Parity status: pinned by the CPU tests (zero and one-bit
 * encoders against their closed forms, the linear decoder's minimiser,
 * J = dx sum f B, and u1 as the minimiser of J over u1).
 * ------------------------------------------------------------------------ */

/* Density of w ~ U(-1, 1): 1/2 on the closed interval |t| <= 1, else 0.
 * (The interval's end points carry no probability; taking them in is a
 * reading, and it decides which grid nodes a window holds.) */
static double orc_box(double t) { return fabs(t) <= 1.0 ? 0.5 : 0.0; }

/* B(u; x) = L_0(u, x) / f(x) for the coding objective (Section III-A,
 * marginal cost C_0): lam u^2 + integral over y of p_w(y - u)(u1(y) - x)^2,
 * by the rectangle rule over every y node in index order. */
double orc_cd_B(const orc_problem* p, double lam, const double* u1, double x, double u) {
  double dy = (p->y_hi - p->y_lo) / (double)(p->n_y - 1);
  double s = 0.0;
  for (int64_t j = 0; j < p->n_y; ++j) {
    double y = orc_node(p->y_lo, p->y_hi, p->n_y, j);
    double e = u1[j] - x;
    s += orc_box(y - u) * e * e;
  }
  return lam * u * u + dy * s;
}

/* L_0(u; x_i) = f_i B(u; x_i) for candidates u [n_x][n_cand]. */
void orc_cd_marginal_cost(const orc_problem* p, double lam, const double* u1, const double* u,
                          int64_t n_cand, double* out) {
  double* f = (double*)malloc(sizeof(double) * (size_t)p->n_x);
  orc_prior(p, f, NULL);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < p->n_x; ++i) {
    double x = orc_node(p->x_lo, p->x_hi, p->n_x, i);
    for (int64_t c = 0; c < n_cand; ++c)
      out[i * n_cand + c] = f[i] * orc_cd_B(p, lam, u1, x, u[i * n_cand + c]);
  }
  free(f);
}

/* The coarse-to-fine u0 update of the Witsenhausen case with the coding
 * B: the same levels, selection rule and incumbent comparison. */
void orc_cd_argmin(const orc_problem* p, double lam, const orc_search* s, const double* u1,
                   const double* u0_in, const int64_t* rows, int64_t n_rows,
                   double* u0_out, double* B_out) {
  orc_argmin_model(p, s, u1, u0_in, rows, n_rows, u0_out, B_out, 1, lam, NULL);
}

/* Second controller by its closed form, the conditional mean
 * u1(y_j) = E[x0 | x1 = y_j] = sum_i f_i p_w(y_j - u0_i) x_i / sum_i f_i p_w(y_j - u0_i),
 * the minimiser of the discrete marginal cost C_1(v, y_j).  Where no node
 * has |y_j - u0_i| <= 1 the ratio is undefined (such y_j carry no
 * probability): u1_j = 0 there, a reading.  rows as in orc_update_u1. */
void orc_cd_update_u1(const orc_problem* p, const double* u0, const int64_t* rows,
                      int64_t n_rows, double* u1_out) {
  double* f = (double*)malloc(sizeof(double) * (size_t)p->n_x);
  orc_prior(p, f, NULL);
  int64_t n = rows ? n_rows : p->n_y;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < n; ++r) {
    int64_t j = rows ? rows[r] : r;
    double y = orc_node(p->y_lo, p->y_hi, p->n_y, j);
    double num = 0.0, den = 0.0;
    for (int64_t i = 0; i < p->n_x; ++i) {
      double wgt = f[i] * orc_box(y - u0[i]);
      num += wgt * orc_node(p->x_lo, p->x_hi, p->n_x, i);
      den += wgt;
    }
    u1_out[r] = den > 0.0 ? num / den : 0.0;
  }
  free(f);
}

/* Objective of Section V-B by the rectangle rule:
 * J = dx * sum_i f_i [lam u0_i^2 + dy * sum_j p_w(y_j - u0_i)(u1_j - x_i)^2]. */
double orc_cd_objective(const orc_problem* p, double lam, const double* u0, const double* u1) {
  double dx = (p->x_hi - p->x_lo) / (double)(p->n_x - 1);
  double dy = (p->y_hi - p->y_lo) / (double)(p->n_y - 1);
  double* f = (double*)malloc(sizeof(double) * (size_t)p->n_x);
  double* row = (double*)malloc(sizeof(double) * (size_t)p->n_x);
  orc_prior(p, f, NULL);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < p->n_x; ++i) {
    double x = orc_node(p->x_lo, p->x_hi, p->n_x, i);
    double s = 0.0;
    for (int64_t j = 0; j < p->n_y; ++j) {
      double y = orc_node(p->y_lo, p->y_hi, p->n_y, j);
      double e = u1[j] - x;
      s += orc_box(y - u0[i]) * e * e;
    }
    row[i] = f[i] * (lam * u0[i] * u0[i] + dy * s);
  }
  double J = 0.0;
  for (int64_t i = 0; i < p->n_x; ++i) J += row[i];
  free(f);
  free(row);
  return dx * J;
}

/* The solve loop of orc_solve for the coding problem. */
void orc_cd_solve(const orc_problem* p, double lam, const orc_search* s, int32_t iters,
                  const double* u0_init, double* u0_out, double* u1_out, double* J_hist) {
  double* u0 = (double*)malloc(sizeof(double) * (size_t)p->n_x);
  double* nxt = (double*)malloc(sizeof(double) * (size_t)p->n_x);
  memcpy(u0, u0_init, sizeof(double) * (size_t)p->n_x);
  orc_cd_update_u1(p, u0, NULL, 0, u1_out);
  J_hist[0] = orc_cd_objective(p, lam, u0, u1_out);
  for (int32_t t = 1; t <= iters; ++t) {
    orc_cd_argmin(p, lam, s, u1_out, u0, NULL, 0, nxt, NULL);
    memcpy(u0, nxt, sizeof(double) * (size_t)p->n_x);
    orc_cd_update_u1(p, u0, NULL, 0, u1_out);
    J_hist[t] = orc_cd_objective(p, lam, u0, u1_out);
  }
  memcpy(u0_out, u0, sizeof(double) * (size_t)p->n_x);
  free(u0);
  free(nxt);
}

/* ------------------------------------------------------------------------
 * Two-dimensional Witsenhausen counterexample (Section V-D): x0 in R^2 with
 * both coordinates independent draws of the prior above, x1 = x0 + u0(x0),
 * y1 = x1 + w with w ~ N(0, I_2), x2 = x1 - u1(y1),
 * J = 1/2 E[k^2 |u0(x0)|^2 + |x2|^2].
 * Grids are tensor products of the 1-D grids above: x node (i1, i2) at
 * index i1 * n_x + i2, y node (j1, j2) at j1 * n_y + j2; vector fields are
 * stored as two planes (first coordinates, then second).  Rectangle rule
 * with weights dx^2 and dy^2.  Parity status: pinned by the CPU tests
 * (separable inputs reduce every function to the 1-D oracle, a closed form
 * for the affine controllers, symmetry).
 * ------------------------------------------------------------------------ */

/* B(u; x) = L_0(u, x) / f(x) for the 2-D objective: 1/2 [k^2 |u|^2 +
 * sum over every y node of dy^2 phi(y1 - z1) phi(y2 - z2) |z - u1(y)|^2],
 * z = x + u; u1 is [2][n_y * n_y]. */
double orc2_B(const orc_problem* p, const double* u1, double x1, double x2, double ua, double ub) {
  double dy = (p->y_hi - p->y_lo) / (double)(p->n_y - 1);
  int64_t ny = p->n_y, nn = ny * ny;
  double z1 = x1 + ua, z2 = x2 + ub;
  double s = 0.0;
  for (int64_t j1 = 0; j1 < ny; ++j1) {
    double g1 = orc_phi(orc_node(p->y_lo, p->y_hi, ny, j1) - z1);
    for (int64_t j2 = 0; j2 < ny; ++j2) {
      double g2 = orc_phi(orc_node(p->y_lo, p->y_hi, ny, j2) - z2);
      double e1 = z1 - u1[j1 * ny + j2];
      double e2 = z2 - u1[nn + j1 * ny + j2];
      s += g1 * g2 * (e1 * e1 + e2 * e2);
    }
  }
  return 0.5 * (p->k * p->k * (ua * ua + ub * ub) + dy * dy * s);
}

/* Prior density of x0 at every 2-D node: f(x1) f(x2). */
static void orc2_prior(const orc_problem* p, double* f2) {
  int64_t n = p->n_x;
  double* f = (double*)malloc(sizeof(double) * (size_t)n);
  orc_prior(p, f, NULL);
  for (int64_t i1 = 0; i1 < n; ++i1)
    for (int64_t i2 = 0; i2 < n; ++i2) f2[i1 * n + i2] = f[i1] * f[i2];
  free(f);
}

/* L_0 = f B for candidates u [2][n_x^2][n_cand] (first coordinates, then
 * second). */
void orc2_marginal_cost(const orc_problem* p, const double* u1, const double* u, int64_t n_cand,
                        double* out) {
  int64_t n = p->n_x, nn = n * n;
  double* f2 = (double*)malloc(sizeof(double) * (size_t)nn);
  orc2_prior(p, f2);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < nn; ++i) {
    double x1 = orc_node(p->x_lo, p->x_hi, n, i / n), x2 = orc_node(p->x_lo, p->x_hi, n, i % n);
    for (int64_t c = 0; c < n_cand; ++c)
      out[i * n_cand + c] =
          f2[i] * orc2_B(p, u1, x1, x2, u[i * n_cand + c], u[nn * n_cand + i * n_cand + c]);
  }
  free(f2);
}

/* Selection among 2-D candidates: ties within the relative band tau of the
 * minimum; the one nearest the incumbent (squared Euclidean distance) wins,
 * then the smaller first coordinate, then the smaller second, then the
 * earlier index. */
static int orc2_select(int n, const double* ca, const double* cb, const double* B, double ia, double ib,
                       double tau) {
  double m = B[0];
  for (int s = 1; s < n; ++s)
    if (B[s] < m) m = B[s];
  double thr = m * (1.0 + tau);
  int best = -1;
  double bd = 0.0;
  for (int s = 0; s < n; ++s) {
    if (!(B[s] <= thr)) continue;
    double da = ca[s] - ia, db = cb[s] - ib;
    double d = da * da + db * db;
    if (best < 0 || d < bd || (d == bd && (ca[s] < ca[best] || (ca[s] == ca[best] && cb[s] < cb[best])))) {
      best = s;
      bd = d;
    }
  }
  return best;
}

/* Coarse-to-fine search in 2-D: level 0 is the K x K tensor grid on
 * [u_lo, u_hi]^2 (candidate q1 * K + q2 at (u_lo + q1 h0, u_lo + q2 h0));
 * level l the K x K grid on the bracket c* -/+ h_{l-1} in each coordinate,
 * clamped, the best so far carried as index K^2; the incumbent compared
 * last.  Same spacings as the 1-D search. */
static void orc2_argmin_point(const orc_problem* p, const orc_search* s, const double* u1,
                              const double* h, double x1, double x2, double ia, double ib,
                              double* oa, double* ob, double* oB) {
  int K = s->cands, KK = K * K;
  double* ca = (double*)malloc(sizeof(double) * (size_t)(KK + 1));
  double* cb = (double*)malloc(sizeof(double) * (size_t)(KK + 1));
  double* B = (double*)malloc(sizeof(double) * (size_t)(KK + 1));
  double sa = 0.0, sb = 0.0, sB = 0.0;
  for (int l = 0; l < s->levels; ++l) {
    for (int q1 = 0; q1 < K; ++q1)
      for (int q2 = 0; q2 < K; ++q2) {
        int q = q1 * K + q2;
        if (l == 0) {
          ca[q] = s->u_lo + (double)q1 * h[0];
          cb[q] = s->u_lo + (double)q2 * h[0];
        } else {
          ca[q] = orc_clamp(sa - h[l - 1] + (double)q1 * h[l], s->u_lo, s->u_hi);
          cb[q] = orc_clamp(sb - h[l - 1] + (double)q2 * h[l], s->u_lo, s->u_hi);
        }
        B[q] = orc2_B(p, u1, x1, x2, ca[q], cb[q]);
      }
    int n = KK;
    if (l > 0) {
      ca[KK] = sa;
      cb[KK] = sb;
      B[KK] = sB;
      n = KK + 1;
    }
    int b = orc2_select(n, ca, cb, B, ia, ib, orc_tau(s));
    sa = ca[b];
    sb = cb[b];
    sB = B[b];
  }
  ca[0] = sa;
  cb[0] = sb;
  B[0] = sB;
  ca[1] = ia;
  cb[1] = ib;
  B[1] = orc2_B(p, u1, x1, x2, ia, ib);
  int b = orc2_select(2, ca, cb, B, ia, ib, orc_tau(s));
  *oa = ca[b];
  *ob = cb[b];
  if (oB) *oB = B[b];
  free(ca);
  free(cb);
  free(B);
}

/* One u0 update of the listed 2-D points (rows == NULL: all n_x^2);
 * u0_in is [2][n_x^2], u0_out [2][n_rows], B_out [n_rows]. */
void orc2_argmin(const orc_problem* p, const orc_search* s, const double* u1, const double* u0_in,
                 const int64_t* rows, int64_t n_rows, double* u0_out, double* B_out) {
  double h[64];
  orc_spacings(s, h);
  int64_t n = p->n_x, nn = n * n;
  int64_t m = rows ? n_rows : nn;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t r = 0; r < m; ++r) {
    int64_t i = rows ? rows[r] : r;
    double x1 = orc_node(p->x_lo, p->x_hi, n, i / n), x2 = orc_node(p->x_lo, p->x_hi, n, i % n);
    double Bv;
    orc2_argmin_point(p, s, u1, h, x1, x2, u0_in[i], u0_in[nn + i], &u0_out[r], &u0_out[m + r], &Bv);
    if (B_out) B_out[r] = Bv;
  }
}

/* Second controller by its closed form, the conditional mean of x1 given
 * y1 = y_j, with the weights max-shifted per y node as in orc_update_u1:
 * l_ij = log f_i - |y_j - x1_i|^2 / 2.  u1_out is [2][n_rows]. */
void orc2_update_u1(const orc_problem* p, const double* u0, const int64_t* rows, int64_t n_rows,
                    double* u1_out) {
  int64_t n = p->n_x, nn = n * n, ny = p->n_y;
  double* lf = (double*)malloc(sizeof(double) * (size_t)n);
  double* lf2 = (double*)malloc(sizeof(double) * (size_t)nn);
  double* xa = (double*)malloc(sizeof(double) * (size_t)nn);
  double* xb = (double*)malloc(sizeof(double) * (size_t)nn);
  orc_prior(p, NULL, lf);
  for (int64_t i = 0; i < nn; ++i) {
    lf2[i] = lf[i / n] + lf[i % n];
    xa[i] = orc_node(p->x_lo, p->x_hi, n, i / n) + u0[i];
    xb[i] = orc_node(p->x_lo, p->x_hi, n, i % n) + u0[nn + i];
  }
  int64_t m = rows ? n_rows : ny * ny;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t r = 0; r < m; ++r) {
    int64_t j = rows ? rows[r] : r;
    double ya = orc_node(p->y_lo, p->y_hi, ny, j / ny), yb = orc_node(p->y_lo, p->y_hi, ny, j % ny);
    double M = -INFINITY;
    for (int64_t i = 0; i < nn; ++i) {
      double da = ya - xa[i], db = yb - xb[i];
      double l = lf2[i] - 0.5 * (da * da + db * db);
      if (l > M) M = l;
    }
    double na = 0.0, nb = 0.0, den = 0.0;
    for (int64_t i = 0; i < nn; ++i) {
      double da = ya - xa[i], db = yb - xb[i];
      double e = exp(lf2[i] - 0.5 * (da * da + db * db) - M);
      na += xa[i] * e;
      nb += xb[i] * e;
      den += e;
    }
    u1_out[r] = na / den;
    u1_out[m + r] = nb / den;
  }
  free(lf);
  free(lf2);
  free(xa);
  free(xb);
}

/* J = dx^2 sum_i f_i B(u0_i; x_i) for the 2-D problem. */
double orc2_objective(const orc_problem* p, const double* u0, const double* u1) {
  int64_t n = p->n_x, nn = n * n;
  double dx = (p->x_hi - p->x_lo) / (double)(n - 1);
  double* f2 = (double*)malloc(sizeof(double) * (size_t)nn);
  double* row = (double*)malloc(sizeof(double) * (size_t)nn);
  orc2_prior(p, f2);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < nn; ++i) {
    double x1 = orc_node(p->x_lo, p->x_hi, n, i / n), x2 = orc_node(p->x_lo, p->x_hi, n, i % n);
    row[i] = f2[i] * orc2_B(p, u1, x1, x2, u0[i], u0[nn + i]);
  }
  double J = 0.0;
  for (int64_t i = 0; i < nn; ++i) J += row[i];
  free(f2);
  free(row);
  return dx * dx * J;
}

/* The solve loop of orc_solve in 2-D; u0 and u1 are two planes each. */
void orc2_solve(const orc_problem* p, const orc_search* s, int32_t iters, const double* u0_init,
                double* u0_out, double* u1_out, double* J_hist) {
  int64_t nn = p->n_x * p->n_x;
  double* u0 = (double*)malloc(sizeof(double) * (size_t)(2 * nn));
  double* nxt = (double*)malloc(sizeof(double) * (size_t)(2 * nn));
  memcpy(u0, u0_init, sizeof(double) * (size_t)(2 * nn));
  orc2_update_u1(p, u0, NULL, 0, u1_out);
  J_hist[0] = orc2_objective(p, u0, u1_out);
  for (int32_t t = 1; t <= iters; ++t) {
    orc2_argmin(p, s, u1_out, u0, NULL, 0, nxt, NULL);
    memcpy(u0, nxt, sizeof(double) * (size_t)(2 * nn));
    orc2_update_u1(p, u0, NULL, 0, u1_out);
    J_hist[t] = orc2_objective(p, u0, u1_out);
  }
  memcpy(u0_out, u0, sizeof(double) * (size_t)(2 * nn));
  free(u0);
  free(nxt);
}

/* ------------------------------------------------------------------------
 * The paper's generic solver (Algorithm 1, Sections III-B to III-D) on the
 * Witsenhausen instance with its two controllers: u_0 on the x grid and u_1
 * on the y grid, each improved by local updates (modified Newton on its
 * marginal cost) and by partial exhaustion over the values the controller
 * takes on the neighbouring grid nodes (the domain-ball candidate set of
 * Eq. (2)), with the iterations of each round shared between the two
 * methods by their last improvements (adaptive minimisation).
 *
 * Marginal costs.  C_0(u, x_i) = f_i B(u; x_i) with B as in orc_B.
 * C_1(u, y_j) = dx sum_i f_i phi(y_j - x1_i) (x1_i - u)^2, the integrand of
 * J in y_1 (so J = dx sum f k^2 u0^2 + dy sum_j C_1(u1_j, y_j)).
 *
 * Readings where the paper is silent or garbled:
 *  - The local update of u_0 works on B = C_0 / f (f > 0): the Newton step
 *    is the same, and the gradient step u - tau B'(u) does not vanish where
 *    f underflows; tau (the "given step size") is a parameter.  No range
 *    is imposed on u.
 *  - C_1 is quadratic in u with C_1'' > 0, so its Newton step is taken as
 *    written, u - C_1'/C_1'', with the weights f_i phi max-shifted per y_j:
 *    the factor cancels in the step.
 *  - Partial exhaustion compares the candidates {u_m at the nodes within r
 *    of the point} (the point's own value among them) by the selection rule
 *    of the coarse-to-fine search (relative tie band, nearest to the
 *    current value, then the smaller u); all points of one controller are
 *    updated from the same previous array (the parallel form of Section
 *    IV-A).  For u_1 the candidates are compared by C_1 with the same
 *    max-shifted weights (a positive factor per y_j changes neither the
 *    order nor the relative band).
 *  - The improvement of a phase is |J before the phase - J after it| (the
 *    printed update subtracts J from the previous improvement); the first
 *    allocation is N_L = floor(N/2), N_P = N - N_L, and an allocation with
 *    I_L + I_P = 0 keeps the previous one.
 *  - The loop stops when I_L + I_P <= p or after max_rounds rounds.
 * Parity status: pinned by the CPU tests (derivatives against the closed
 * form with a linear u_1 and against central differences, one Newton step
 * onto the minimiser of the convex case, the u_1 step equal to the closed
 * form, partial exhaustion never raising J and undoing an isolated spike,
 * the allocation rule on hand-made improvements, and a 40-digit
 * evaluation of one local update and one partial exhaustion).
 * ------------------------------------------------------------------------ */

/* B(u; x) and its first two derivatives in u (the local update's C_0' and
 * C_0'' divided by f).  With z = x + u, t_j = (y_j - z) / s^2 and
 * e_j = z - u1_j: d phi_s(y_j - z)/dz = t_j phi_s, so
 *   B'  = 2 k^2 u + dy sum_j phi_s (t_j e_j^2 + 2 e_j),
 *   B'' = 2 k^2   + dy sum_j phi_s ((t_j^2 - 1/s^2) e_j^2 + 4 t_j e_j + 2). */
void orc_B_derivs(const orc_problem* p, const double* u1, double x, double u, double* B, double* B1,
                  double* B2) {
  double dy = (p->y_hi - p->y_lo) / (double)(p->n_y - 1);
  double sw = orc_noise_sd(p);
  double is2 = 1.0 / (sw * sw);
  double z = x + u;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t j = 0; j < p->n_y; ++j) {
    double y = orc_node(p->y_lo, p->y_hi, p->n_y, j);
    double ph = orc_phi_s(y - z, sw);
    double t = (y - z) * is2;
    double e = z - u1[j];
    s0 += ph * e * e;
    s1 += ph * (t * e * e + 2.0 * e);
    s2 += ph * ((t * t - is2) * e * e + 4.0 * t * e + 2.0);
  }
  double k2 = p->k * p->k;
  if (B) *B = k2 * u * u + dy * s0;
  if (B1) *B1 = 2.0 * k2 * u + dy * s1;
  if (B2) *B2 = 2.0 * k2 + dy * s2;
}

/* Local update of u_0 (Section III-D): Newton where the curvature is
 * positive, else a gradient step of size tau. */
void orc_alg1_local_u0(const orc_problem* p, double tau, const double* u1, const double* u0_in,
                       const int64_t* rows, int64_t n_rows, double* u0_out) {
  int64_t n = rows ? n_rows : p->n_x;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < n; ++r) {
    int64_t i = rows ? rows[r] : r;
    double x = orc_node(p->x_lo, p->x_hi, p->n_x, i);
    double u = u0_in[i], B1, B2;
    orc_B_derivs(p, u1, x, u, NULL, &B1, &B2);
    u0_out[r] = B2 > 0.0 ? u - B1 / B2 : u - tau * B1;
  }
}

/* Max-shifted weights of C_1 at y_j: w_i = exp(l_ij - M_j), l_ij = log f_i
 * - (y_j - x1_i)^2 / (2 s^2), M_j = max_i l_ij (as in orc_update_u1). */
static void orc_c1_weights(const orc_problem* p, const double* logf, const double* x1, double y, double* w) {
  const double sw = orc_noise_sd(p);
  double M = -INFINITY;
  for (int64_t i = 0; i < p->n_x; ++i) {
    double d = (y - x1[i]) / sw;
    double l = logf[i] - 0.5 * d * d;
    if (l > M) M = l;
  }
  for (int64_t i = 0; i < p->n_x; ++i) {
    double d = (y - x1[i]) / sw;
    w[i] = exp(logf[i] - 0.5 * d * d - M);
  }
}

/* Local update of u_1: the Newton step u - C_1'(u)/C_1''(u) with
 * C_1' = -2 sum w (x1 - u) and C_1'' = 2 sum w (common factors dropped). */
void orc_alg1_local_u1(const orc_problem* p, const double* u0, const double* u1_in, const int64_t* rows,
                       int64_t n_rows, double* u1_out) {
  double* logf = (double*)malloc(sizeof(double) * (size_t)p->n_x);
  double* x1 = (double*)malloc(sizeof(double) * (size_t)p->n_x);
  orc_prior(p, NULL, logf);
  for (int64_t i = 0; i < p->n_x; ++i) x1[i] = orc_node(p->x_lo, p->x_hi, p->n_x, i) + u0[i];
  int64_t n = rows ? n_rows : p->n_y;
#pragma omp parallel
  {
    double* w = (double*)malloc(sizeof(double) * (size_t)p->n_x);
#pragma omp for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
      int64_t j = rows ? rows[r] : r;
      double y = orc_node(p->y_lo, p->y_hi, p->n_y, j);
      double u = u1_in[j];
      orc_c1_weights(p, logf, x1, y, w);
      double c1 = 0.0, c2 = 0.0;
      for (int64_t i = 0; i < p->n_x; ++i) {
        c1 += -2.0 * w[i] * (x1[i] - u);
        c2 += 2.0 * w[i];
      }
      u1_out[r] = u - c1 / c2;
    }
    free(w);
  }
  free(logf);
  free(x1);
}

/* Partial exhaustion of u_0 over the values at the nodes within r of x_i. */
void orc_alg1_pe_u0(const orc_problem* p, double tie, int32_t r, const double* u1, const double* u0_in,
                    const int64_t* rows, int64_t n_rows, double* u0_out) {
  int64_t n = rows ? n_rows : p->n_x;
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < n; ++q) {
    int64_t i = rows ? rows[q] : q;
    double x = orc_node(p->x_lo, p->x_hi, p->n_x, i);
    double c[64], B[64];
    int m = 0;
    for (int64_t k = i - r; k <= i + r; ++k) {
      if (k < 0 || k >= p->n_x) continue;
      c[m] = u0_in[k];
      B[m] = orc_B(p, u1, x, c[m]);
      ++m;
    }
    u0_out[q] = c[orc_select(m, c, B, u0_in[i], tie)];
  }
}

/* Partial exhaustion of u_1 over the values at the nodes within r of y_j,
 * compared by C_1(u, y_j) with max-shifted weights. */
void orc_alg1_pe_u1(const orc_problem* p, double tie, int32_t r, const double* u0, const double* u1_in,
                    const int64_t* rows, int64_t n_rows, double* u1_out) {
  double* logf = (double*)malloc(sizeof(double) * (size_t)p->n_x);
  double* x1 = (double*)malloc(sizeof(double) * (size_t)p->n_x);
  orc_prior(p, NULL, logf);
  for (int64_t i = 0; i < p->n_x; ++i) x1[i] = orc_node(p->x_lo, p->x_hi, p->n_x, i) + u0[i];
  int64_t n = rows ? n_rows : p->n_y;
#pragma omp parallel
  {
    double* w = (double*)malloc(sizeof(double) * (size_t)p->n_x);
#pragma omp for schedule(static)
    for (int64_t q = 0; q < n; ++q) {
      int64_t j = rows ? rows[q] : q;
      double y = orc_node(p->y_lo, p->y_hi, p->n_y, j);
      orc_c1_weights(p, logf, x1, y, w);
      double c[64], C[64];
      int m = 0;
      for (int64_t k = j - r; k <= j + r; ++k) {
        if (k < 0 || k >= p->n_y) continue;
        c[m] = u1_in[k];
        double s = 0.0;
        for (int64_t i = 0; i < p->n_x; ++i) {
          double e = x1[i] - c[m];
          s += w[i] * e * e;
        }
        C[m] = s;
        ++m;
      }
      u1_out[q] = c[orc_select(m, c, C, u1_in[j], tie)];
    }
    free(w);
  }
  free(logf);
  free(x1);
}

/* Adaptive minimisation (the last line of Algorithm 1's loop): the N
 * iterations of the next round shared in proportion to the improvements,
 * each method keeping at least one. */
void orc_alg1_allocate(int32_t N, double IL, double IP, int32_t* NL, int32_t* NP) {
  if (IL + IP > 0.0) {
    double a = floor(IL * (double)N / (IL + IP));
    int32_t v = (int32_t)a;
    if (v < 1) v = 1;
    if (v > N - 1) v = N - 1;
    *NL = v;
  }
  *NP = N - *NL;
}

typedef struct {
  int32_t N;          /* iterations per round */
  int32_t r;          /* partial-exhaustion radius in grid nodes */
  double p;           /* precision: stop when I_L + I_P <= p */
  double tau;         /* gradient step size of the local update */
  double tie_rel64;   /* relative tie band of partial exhaustion (0: ORC_TAU64) */
  int32_t max_rounds; /* cap on rounds */
  int32_t pad_;
} orc_alg1_params;

/* Algorithm 1.  J_log receives J after initialisation and after each phase
 * ([1 + 2 rounds]); NL_log the local-update iterations of each round.
 * Returns the number of rounds run. */
int32_t orc_alg1_solve(const orc_problem* p, const orc_alg1_params* a, const double* u0_init,
                       const double* u1_init, double* u0_out, double* u1_out, double* J_log, int32_t* NL_log) {
  const double tie = a->tie_rel64 > 0.0 ? a->tie_rel64 : ORC_TAU64;
  double* u0 = (double*)malloc(sizeof(double) * (size_t)p->n_x);
  double* u1 = (double*)malloc(sizeof(double) * (size_t)p->n_y);
  double* t0 = (double*)malloc(sizeof(double) * (size_t)p->n_x);
  double* t1 = (double*)malloc(sizeof(double) * (size_t)p->n_y);
  memcpy(u0, u0_init, sizeof(double) * (size_t)p->n_x);
  memcpy(u1, u1_init, sizeof(double) * (size_t)p->n_y);
  double Jc = orc_objective(p, u0, u1);
  J_log[0] = Jc;
  double IL = a->p, IP = a->p;
  int32_t NL = a->N / 2, NP = a->N - NL;
  int32_t rounds = 0;
  while (IL + IP > a->p && rounds < a->max_rounds) {
    NL_log[rounds] = NL;
    double Jprev = Jc;
    for (int32_t it = 0; it < NL; ++it) {
      orc_alg1_local_u0(p, a->tau, u1, u0, NULL, 0, t0);
      memcpy(u0, t0, sizeof(double) * (size_t)p->n_x);
      orc_alg1_local_u1(p, u0, u1, NULL, 0, t1);
      memcpy(u1, t1, sizeof(double) * (size_t)p->n_y);
    }
    Jc = orc_objective(p, u0, u1);
    IL = fabs(Jprev - Jc);
    J_log[1 + 2 * rounds] = Jc;
    Jprev = Jc;
    for (int32_t it = 0; it < NP; ++it) {
      orc_alg1_pe_u0(p, tie, a->r, u1, u0, NULL, 0, t0);
      memcpy(u0, t0, sizeof(double) * (size_t)p->n_x);
      orc_alg1_pe_u1(p, tie, a->r, u0, u1, NULL, 0, t1);
      memcpy(u1, t1, sizeof(double) * (size_t)p->n_y);
    }
    Jc = orc_objective(p, u0, u1);
    IP = fabs(Jprev - Jc);
    J_log[2 + 2 * rounds] = Jc;
    orc_alg1_allocate(a->N, IL, IP, &NL, &NP);
    ++rounds;
  }
  memcpy(u0_out, u0, sizeof(double) * (size_t)p->n_x);
  memcpy(u1_out, u1, sizeof(double) * (size_t)p->n_y);
  free(u0);
  free(u1);
  free(t0);
  free(t1);
  return rounds;
}
