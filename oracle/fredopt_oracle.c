/*
 * FP64 CPU oracle for superiorized dose / LETd feasibility seeking
 * (Borys et al., arXiv 2509.20012, Section 2.4.3, Figs. 2-3, Eq. 2).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the HIP
 * path is checked against.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or helper
 * with the HIP library: it reads the same FP32 input arrays (promoted to FP64 by
 * its Python wrapper) and computes everything from the definitions below.
 *
 * Notation: R voxel rows, C beamlet columns, CSR matrices D (dose per unit fluence)
 * and L (LET-weighted dose, the LETd numerator of Eq. 1) with a shared pattern.
 *   d = D x, l = L x, LETd_i = l_i / d_i (0 where d_i = 0), cDL_i = c l_i.
 * Constraint kinds per row (bit mask), each a half-space <a, x> (<= or >=) b:
 *   DOSE_LO  a = D_i,             >= dose_lo_i    (Fig. 2, dose block)
 *   DOSE_HI  a = D_i,             <= dose_hi_i
 *   CDL_LO   a = c L_i,           >= cdl_lo_i     (Fig. 2, cDLET block)
 *   CDL_HI   a = c L_i,           <= cdl_hi_i
 *   LETD_HI  a = L_i - T_i D_i,   <= 0            (LETd_i <= T_i, linearised)
 * Objective terms (Eq. 2): OBJ_DOSE rows w_obj (Dhat - d)^2, OBJ_CDL rows
 * w_obj (cDLhat - c l)^2 as printed, or, with the one-sided reading of the OAR
 * term, w_obj (cDLhat - c l)^2 only where c l > cDLhat (0 below the target).
 *
 * Parity is pinned by the CPU tests (dense brute force, closed forms, invariants);
 * nothing here is compared against itself.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define K_DOSE_LO (1u << 0)
#define K_DOSE_HI (1u << 1)
#define K_CDL_LO (1u << 2)
#define K_CDL_HI (1u << 3)
#define K_LETD_HI (1u << 4)
#define K_OBJ_DOSE (1u << 5)
#define K_OBJ_CDL (1u << 6)

/* a constraint whose normal has squared norm at or below this fraction of its
 * scale is degenerate and skipped (reading of the paper's silence on zero rows) */
#define DEGENERATE_REL 1e-12
/* the step-size search gives up once alpha^s falls below this (reading of Fig. 3's
 * unbounded inner loop) */
#define BETA_FLOOR 1e-300

typedef struct {
  int64_t R, C;
  const int64_t *row_ptr;
  const int32_t *col;
  const double *dv, *lv;
  /* CSC copy (built here) for the transposed products */
  int64_t *col_ptr;
  int32_t *row;
  double *cdv, *clv;
} orc_mat;

typedef struct {
  const uint16_t *kind;
  const double *dose_lo, *dose_hi, *cdl_lo, *cdl_hi, *letd_max;
  const double *w_feas, *w_obj, *dose_target, *cdl_target;
  double c;
  int32_t objective;     /* 0: Eq. (2) as printed, 1: OAR term one-sided (above cDLhat) */
} orc_problem;

typedef struct {
  double lambda, alpha, eta;
  int32_t reductions_n;
  int32_t normalization; /* 0: convex over all constraints, 1: convex over violated, 2: raw */
  int32_t line_search;   /* 0: literal cost comparison, 1: exact quadratic identity */
  int32_t unit_direction; /* 0: perturb along grad chi^2 as printed, 1: grad / ||grad|| */
} orc_params;

typedef struct {
  int64_t n_accepted;     /* perturbations accepted in this outer iteration */
  int64_t n_trials;       /* step sizes tried */
  int64_t n_violated;     /* violated constraints at the AMS input point */
  double beta_last, cost_before, cost_after_perturb, proximity, grad_sq, q_last;
  int32_t capped;         /* 1 if a step-size search hit BETA_FLOOR */
} orc_iter_info;

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the parallel loops that follow (n >= 1); used to time the oracle on one
 * host core next to all of them. */
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ---------------------------------------------------------------- matrices ---- */

/* Counting-sort transpose: within each column rows come out ascending. */
int orc_mat_init(orc_mat *m, int64_t R, int64_t C, const int64_t *row_ptr,
                 const int32_t *col, const double *dv, const double *lv) {
  m->R = R; m->C = C; m->row_ptr = row_ptr; m->col = col; m->dv = dv; m->lv = lv;
  int64_t nnz = row_ptr[R];
  m->col_ptr = (int64_t *)calloc((size_t)C + 1, sizeof(int64_t));
  m->row = (int32_t *)malloc((size_t)(nnz ? nnz : 1) * sizeof(int32_t));
  m->cdv = (double *)malloc((size_t)(nnz ? nnz : 1) * sizeof(double));
  m->clv = (double *)malloc((size_t)(nnz ? nnz : 1) * sizeof(double));
  if (!m->col_ptr || !m->row || !m->cdv || !m->clv) return -1;
  for (int64_t k = 0; k < nnz; ++k) m->col_ptr[col[k] + 1]++;
  for (int64_t j = 0; j < C; ++j) m->col_ptr[j + 1] += m->col_ptr[j];
  int64_t *cur = (int64_t *)malloc((size_t)(C ? C : 1) * sizeof(int64_t));
  if (!cur) return -1;
  memcpy(cur, m->col_ptr, (size_t)C * sizeof(int64_t));
  for (int64_t i = 0; i < R; ++i)
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      int64_t p = cur[col[k]]++;
      m->row[p] = (int32_t)i;
      m->cdv[p] = dv[k];
      m->clv[p] = lv[k];
    }
  free(cur);
  return 0;
}

void orc_mat_free(orc_mat *m) {
  free(m->col_ptr); free(m->row); free(m->cdv); free(m->clv);
  m->col_ptr = NULL; m->row = NULL; m->cdv = NULL; m->clv = NULL;
}

/* ---------------------------------------------------------------- products ---- */

/* d = D x and l = L x (the row dot products <D_i, x>, <L_i, x> of Fig. 2). */
void orc_forward(const orc_mat *m, const double *x, double *d, double *l) {
  int64_t i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < m->R; ++i) {
    double sd = 0.0, sl = 0.0;
    for (int64_t k = m->row_ptr[i]; k < m->row_ptr[i + 1]; ++k) {
      sd += m->dv[k] * x[m->col[k]];
      sl += m->lv[k] * x[m->col[k]];
    }
    d[i] = sd;
    l[i] = sl;
  }
}

/* Same products for a subset of rows (spot checks at full size). */
void orc_forward_rows(const orc_mat *m, const double *x, const int64_t *rows, int64_t n,
                      double *d, double *l) {
  int64_t t;
#pragma omp parallel for schedule(static)
  for (t = 0; t < n; ++t) {
    int64_t i = rows[t];
    double sd = 0.0, sl = 0.0;
    for (int64_t k = m->row_ptr[i]; k < m->row_ptr[i + 1]; ++k) {
      sd += m->dv[k] * x[m->col[k]];
      sl += m->lv[k] * x[m->col[k]];
    }
    d[t] = sd;
    l[t] = sl;
  }
}

/* out = D^T ud + L^T ul, each column summed over ascending rows. */
void orc_transposed(const orc_mat *m, const double *ud, const double *ul, double *out) {
  int64_t j;
#pragma omp parallel for schedule(static)
  for (j = 0; j < m->C; ++j) {
    double s = 0.0;
    for (int64_t k = m->col_ptr[j]; k < m->col_ptr[j + 1]; ++k)
      s += m->cdv[k] * ud[m->row[k]] + m->clv[k] * ul[m->row[k]];
    out[j] = s;
  }
}

/* Dose, LETd (Eq. 1 from its additive numerator and denominator, Section 2.2) and
 * cDL = c * dose * LETd = c * l (Section 2.4). */
void orc_dose_let(const orc_mat *m, const double *x, double c, double *d, double *l,
                  double *letd, double *cdl) {
  orc_forward(m, x, d, l);
  for (int64_t i = 0; i < m->R; ++i) {
    if (letd) letd[i] = d[i] > 0.0 ? l[i] / d[i] : 0.0;
    if (cdl) cdl[i] = c * l[i];
  }
}

/* ---------------------------------------------------------------- objective --- */

/* Whether the OAR term of row i counts at residual f = cDLhat - c l: always as Eq. (2)
 * is printed; only above the target (f < 0) in the one-sided reading. */
static int oar_term_on(const orc_problem *p, double f) { return p->objective == 0 || f < 0.0; }

/* Eq. (2): sum over PTV rows of w (Dhat - d)^2 plus over OAR rows of
 * w (cDLhat - c l)^2 (one-sided reading: only rows with c l > cDLhat). */
static double cost_from_dl(const orc_mat *m, const orc_problem *p, const double *d,
                           const double *l) {
  double s = 0.0;
  for (int64_t i = 0; i < m->R; ++i) {
    unsigned k = p->kind[i];
    if (k & K_OBJ_DOSE) {
      double e = p->dose_target[i] - d[i];
      s += p->w_obj[i] * e * e;
    }
    if (k & K_OBJ_CDL) {
      double f = p->cdl_target[i] - p->c * l[i];
      if (oar_term_on(p, f)) s += p->w_obj[i] * f * f;
    }
  }
  return s;
}

double orc_cost(const orc_mat *m, const orc_problem *p, const double *x) {
  double *d = (double *)malloc((size_t)(m->R ? m->R : 1) * sizeof(double));
  double *l = (double *)malloc((size_t)(m->R ? m->R : 1) * sizeof(double));
  orc_forward(m, x, d, l);
  double s = cost_from_dl(m, p, d, l);
  free(d); free(l);
  return s;
}

/* Gradient of Eq. (2): -2 D^T[w (Dhat - d)]_PTV - 2 c L^T[w (cDLhat - c l)]_OAR; in the
 * one-sided reading the OAR rows below their target contribute nothing (the squared
 * hinge is differentiable, with derivative 0 at the target). */
void orc_gradient(const orc_mat *m, const orc_problem *p, const double *x, double *g) {
  int64_t R = m->R;
  double *d = (double *)malloc((size_t)(R ? R : 1) * sizeof(double));
  double *l = (double *)malloc((size_t)(R ? R : 1) * sizeof(double));
  double *ud = (double *)calloc((size_t)(R ? R : 1), sizeof(double));
  double *ul = (double *)calloc((size_t)(R ? R : 1), sizeof(double));
  orc_forward(m, x, d, l);
  for (int64_t i = 0; i < R; ++i) {
    unsigned k = p->kind[i];
    if (k & K_OBJ_DOSE) ud[i] = -2.0 * p->w_obj[i] * (p->dose_target[i] - d[i]);
    if (k & K_OBJ_CDL) {
      double f = p->cdl_target[i] - p->c * l[i];
      if (oar_term_on(p, f)) ul[i] = -2.0 * p->c * p->w_obj[i] * f;
    }
  }
  orc_transposed(m, ud, ul, g);
  free(d); free(l); free(ud); free(ul);
}

/* ------------------------------------------------------------- constraints ---- */

/* Squared norm of the constraint normal a of row i and kind bit, computed directly
 * from the row's entries. *scale receives the quantity DEGENERATE_REL refers to. */
static double normal_sq(const orc_mat *m, const orc_problem *p, int64_t i, unsigned kind,
                        double *scale) {
  double s = 0.0, sd = 0.0, sl = 0.0;
  double T = p->letd_max[i];
  for (int64_t k = m->row_ptr[i]; k < m->row_ptr[i + 1]; ++k) {
    double a;
    if (kind == K_DOSE_LO || kind == K_DOSE_HI) a = m->dv[k];
    else if (kind == K_CDL_LO || kind == K_CDL_HI) a = p->c * m->lv[k];
    else a = m->lv[k] - T * m->dv[k];
    s += a * a;
    sd += m->dv[k] * m->dv[k];
    sl += m->lv[k] * m->lv[k];
  }
  if (kind == K_LETD_HI) *scale = sl + T * T * sd;
  else *scale = s;
  return s;
}

/* Signed violation v of the (row, kind) half-space at the point with row products
 * (di, li): for "<=" v = <a,x> - b where <a,x> > b, for ">=" v = <a,x> - b where
 * <a,x> < b, else 0.  Equality is not a violation (strict tests of Fig. 2). */
static double violation(const orc_problem *p, int64_t i, unsigned kind, double di,
                        double li) {
  double ax;
  switch (kind) {
    case K_DOSE_HI: ax = di; return ax > p->dose_hi[i] ? ax - p->dose_hi[i] : 0.0;
    case K_DOSE_LO: ax = di; return ax < p->dose_lo[i] ? ax - p->dose_lo[i] : 0.0;
    case K_CDL_HI: ax = p->c * li; return ax > p->cdl_hi[i] ? ax - p->cdl_hi[i] : 0.0;
    case K_CDL_LO: ax = p->c * li; return ax < p->cdl_lo[i] ? ax - p->cdl_lo[i] : 0.0;
    case K_LETD_HI: ax = li - p->letd_max[i] * di; return ax > 0.0 ? ax : 0.0;
  }
  return 0.0;
}

static const unsigned KIND_ORDER[5] = {K_DOSE_HI, K_DOSE_LO, K_CDL_HI, K_CDL_LO, K_LETD_HI};

/* Proximity p(y) = 1/2 sum (w_i / W_all) v^2 / ||a||^2 over all constraints, with
 * W_all the sum of w_i over every enabled (row, kind).  Reported, not in the paper. */
double orc_proximity(const orc_mat *m, const orc_problem *p, const double *y,
                     int64_t *n_violated) {
  int64_t R = m->R;
  double *d = (double *)malloc((size_t)(R ? R : 1) * sizeof(double));
  double *l = (double *)malloc((size_t)(R ? R : 1) * sizeof(double));
  orc_forward(m, y, d, l);
  double wall = 0.0, acc = 0.0;
  int64_t nv = 0;
  for (int64_t i = 0; i < R; ++i)
    for (int q = 0; q < 5; ++q) {
      unsigned kb = KIND_ORDER[q];
      if (!(p->kind[i] & kb)) continue;
      wall += p->w_feas[i];
      double v = violation(p, i, kb, d[i], l[i]);
      if (v == 0.0) continue;
      double scale, na = normal_sq(m, p, i, kb, &scale);
      if (!(na > DEGENERATE_REL * scale)) continue;
      acc += p->w_feas[i] * v * v / na;
      nv++;
    }
  free(d); free(l);
  if (n_violated) *n_violated = nv;
  return wall > 0.0 ? 0.5 * acc / wall : 0.0;
}

/* Simultaneous relaxed projection (the parallel form of Fig. 2): at the fixed point
 * y every violated half-space contributes lambda * wt_i * v / ||a||^2 * a, all
 * contributions are summed, and the result is clamped to x >= 0 (Fig. 2, last
 * loop).  wt_i = weight_scale * w_i / W, with W per `normalization`.  Returns the
 * proximity of y. */
double orc_ams_simultaneous(const orc_mat *m, const orc_problem *p, double lambda,
                            double weight_scale, int normalization, const double *y,
                            double *x_out, int64_t *n_violated) {
  int64_t R = m->R, C = m->C;
  double *d = (double *)malloc((size_t)(R ? R : 1) * sizeof(double));
  double *l = (double *)malloc((size_t)(R ? R : 1) * sizeof(double));
  double *cd = (double *)calloc((size_t)(R ? R : 1), sizeof(double));
  double *cl = (double *)calloc((size_t)(R ? R : 1), sizeof(double));
  double *v = (double *)calloc((size_t)(R ? R : 1) * 5, sizeof(double));
  double *na = (double *)calloc((size_t)(R ? R : 1) * 5, sizeof(double));
  double *t = (double *)malloc((size_t)(C ? C : 1) * sizeof(double));
  orc_forward(m, y, d, l);
  double wall = 0.0, wviol = 0.0, prox = 0.0;
  int64_t nv = 0;
  for (int64_t i = 0; i < R; ++i)
    for (int q = 0; q < 5; ++q) {
      unsigned kb = KIND_ORDER[q];
      if (!(p->kind[i] & kb)) continue;
      wall += p->w_feas[i];
      double vi = violation(p, i, kb, d[i], l[i]);
      if (vi == 0.0) continue;
      double scale, n2 = normal_sq(m, p, i, kb, &scale);
      if (!(n2 > DEGENERATE_REL * scale)) continue;
      v[i * 5 + q] = vi;
      na[i * 5 + q] = n2;
      wviol += p->w_feas[i];
      prox += p->w_feas[i] * vi * vi / n2;
      nv++;
    }
  double W = normalization == 0 ? wall : (normalization == 1 ? wviol : 1.0);
  for (int64_t i = 0; i < R; ++i)
    for (int q = 0; q < 5; ++q) {
      double vi = v[i * 5 + q];
      if (vi == 0.0) continue;
      double kappa = lambda * (weight_scale * p->w_feas[i] / W) * vi / na[i * 5 + q];
      unsigned kb = KIND_ORDER[q];
      if (kb == K_DOSE_HI || kb == K_DOSE_LO) cd[i] += kappa;
      else if (kb == K_CDL_HI || kb == K_CDL_LO) cl[i] += p->c * kappa;
      else { cl[i] += kappa; cd[i] -= p->letd_max[i] * kappa; }
    }
  orc_transposed(m, cd, cl, t);
  for (int64_t j = 0; j < C; ++j) {
    double xj = y[j] - t[j];
    x_out[j] = xj > 0.0 ? xj : 0.0;
  }
  free(d); free(l); free(cd); free(cl); free(v); free(na); free(t);
  if (n_violated) *n_violated = nv;
  return wall > 0.0 ? 0.5 * prox / wall : 0.0;
}

/* Block-sequential form of the sweep (Fig. 2 processes one constraint after the
 * other on the current x; the text calls for projections in parallel, and the
 * simultaneous form above takes them all at one x).  Rows are cut into consecutive
 * blocks of block_rows rows; the blocks are taken in ascending order, each as a
 * simultaneous relaxed projection of its own rows' constraints at the current x,
 * with the weights normalised over that block only (convex over its enabled pairs,
 * over its violated pairs, or raw).  x >= 0 is imposed once, after the last block,
 * as Fig. 2 clamps at the end.  One block of R rows is the simultaneous sweep;
 * blocks of one row with one constraint each and raw weights are the sequential
 * sweep of Fig. 2. */
void orc_ams_blocks(const orc_mat *m, const orc_problem *p, double lambda, double weight_scale,
                    int normalization, int64_t block_rows, const double *y, double *x_out) {
  int64_t R = m->R, C = m->C;
  double *x = (double *)malloc((size_t)(C ? C : 1) * sizeof(double));
  double *d = (double *)malloc((size_t)(R ? R : 1) * sizeof(double));
  double *l = (double *)malloc((size_t)(R ? R : 1) * sizeof(double));
  double *cd = (double *)malloc((size_t)(R ? R : 1) * sizeof(double));
  double *cl = (double *)malloc((size_t)(R ? R : 1) * sizeof(double));
  double *t = (double *)malloc((size_t)(C ? C : 1) * sizeof(double));
  memcpy(x, y, (size_t)C * sizeof(double));
  if (block_rows < 1) block_rows = 1;
  for (int64_t b0 = 0; b0 < R; b0 += block_rows) {
    int64_t b1 = b0 + block_rows < R ? b0 + block_rows : R;
    orc_forward(m, x, d, l);
    double wall = 0.0, wviol = 0.0;
    for (int64_t i = b0; i < b1; ++i)
      for (int q = 0; q < 5; ++q) {
        unsigned kb = KIND_ORDER[q];
        if (!(p->kind[i] & kb)) continue;
        wall += p->w_feas[i];
        if (violation(p, i, kb, d[i], l[i]) != 0.0) {
          double scale, n2 = normal_sq(m, p, i, kb, &scale);
          if (n2 > DEGENERATE_REL * scale) wviol += p->w_feas[i];
        }
      }
    double W = normalization == 0 ? wall : (normalization == 1 ? wviol : 1.0);
    memset(cd, 0, (size_t)R * sizeof(double));
    memset(cl, 0, (size_t)R * sizeof(double));
    for (int64_t i = b0; i < b1; ++i)
      for (int q = 0; q < 5; ++q) {
        unsigned kb = KIND_ORDER[q];
        if (!(p->kind[i] & kb)) continue;
        double vi = violation(p, i, kb, d[i], l[i]);
        if (vi == 0.0) continue;
        double scale, n2 = normal_sq(m, p, i, kb, &scale);
        if (!(n2 > DEGENERATE_REL * scale)) continue;
        double kappa = lambda * (weight_scale * p->w_feas[i] / W) * vi / n2;
        if (kb == K_DOSE_HI || kb == K_DOSE_LO) cd[i] += kappa;
        else if (kb == K_CDL_HI || kb == K_CDL_LO) cl[i] += p->c * kappa;
        else { cl[i] += kappa; cd[i] -= p->letd_max[i] * kappa; }
      }
    orc_transposed(m, cd, cl, t);
    for (int64_t j = 0; j < C; ++j) x[j] = x[j] - t[j];
  }
  for (int64_t j = 0; j < C; ++j) x_out[j] = x[j] > 0.0 ? x[j] : 0.0;
  free(x); free(d); free(l); free(cd); free(cl); free(t);
}

/* Row dot product <a, x> for one (row, kind). */
static double row_dot(const orc_mat *m, const orc_problem *p, int64_t i, unsigned kind,
                      const double *x) {
  double s = 0.0, T = p->letd_max[i];
  for (int64_t k = m->row_ptr[i]; k < m->row_ptr[i + 1]; ++k) {
    double a;
    if (kind == K_DOSE_LO || kind == K_DOSE_HI) a = m->dv[k];
    else if (kind == K_CDL_LO || kind == K_CDL_HI) a = p->c * m->lv[k];
    else a = m->lv[k] - T * m->dv[k];
    s += a * x[m->col[k]];
  }
  return s;
}

static void row_axpy(const orc_mat *m, const orc_problem *p, int64_t i, unsigned kind,
                     double coef, double *x) {
  double T = p->letd_max[i];
  for (int64_t k = m->row_ptr[i]; k < m->row_ptr[i + 1]; ++k) {
    double a;
    if (kind == K_DOSE_LO || kind == K_DOSE_HI) a = m->dv[k];
    else if (kind == K_CDL_LO || kind == K_CDL_HI) a = p->c * m->lv[k];
    else a = m->lv[k] - T * m->dv[k];
    x[m->col[k]] -= coef * a;
  }
}

static void seq_check(const orc_mat *m, const orc_problem *p, int64_t i, unsigned kb,
                      double lambda, double weight_scale, double *x) {
  if (!(p->kind[i] & kb)) return;
  double ax = row_dot(m, p, i, kb, x);
  double v;
  switch (kb) {
    case K_DOSE_HI: v = ax > p->dose_hi[i] ? ax - p->dose_hi[i] : 0.0; break;
    case K_DOSE_LO: v = ax < p->dose_lo[i] ? ax - p->dose_lo[i] : 0.0; break;
    case K_CDL_HI: v = ax > p->cdl_hi[i] ? ax - p->cdl_hi[i] : 0.0; break;
    case K_CDL_LO: v = ax < p->cdl_lo[i] ? ax - p->cdl_lo[i] : 0.0; break;
    default: v = ax > 0.0 ? ax : 0.0; break;
  }
  if (v == 0.0) return;
  double scale, n2 = normal_sq(m, p, i, kb, &scale);
  if (!(n2 > DEGENERATE_REL * scale)) return;
  row_axpy(m, p, i, kb, lambda * weight_scale * p->w_feas[i] * v / n2, x);
}

/* Sequential AMS sweep as written in Fig. 2: the dose block visits dose_order
 * (ROIs in listed order, voxels ascending), checking the upper then the lower bound,
 * each on the current fluence; then the cDLET block visits cdl_order checking the
 * cDL upper, cDL lower and LETd bounds; finally the fluence is clamped to >= 0.
 * Every step uses the raw weight lambda * weight_scale * w_i. */
void orc_ams_sequential(const orc_mat *m, const orc_problem *p, double lambda,
                        double weight_scale, const int64_t *dose_order, int64_t n_dose,
                        const int64_t *cdl_order, int64_t n_cdl, double *x) {
  for (int64_t t = 0; t < n_dose; ++t) {
    int64_t i = dose_order[t];
    seq_check(m, p, i, K_DOSE_HI, lambda, weight_scale, x);
    seq_check(m, p, i, K_DOSE_LO, lambda, weight_scale, x);
  }
  for (int64_t t = 0; t < n_cdl; ++t) {
    int64_t i = cdl_order[t];
    seq_check(m, p, i, K_CDL_HI, lambda, weight_scale, x);
    seq_check(m, p, i, K_CDL_LO, lambda, weight_scale, x);
    seq_check(m, p, i, K_LETD_HI, lambda, weight_scale, x);
  }
  for (int64_t j = 0; j < m->C; ++j)
    if (x[j] < 0.0) x[j] = 0.0;
}

/* ------------------------------------------------------------ superiorization -- */

/* One outer iteration k of Fig. 3 (SuperiorDLET), with the perturbed point fed to
 * the feasibility-seeking step:
 *   y = x
 *   repeat reductions_n times:
 *     g = grad chi^2(y); stop perturbing if g = 0
 *     s = s + 1, beta = alpha^s, until chi^2(y - beta g) < chi^2(y); y = y - beta g
 *   x = AMS(y) with weights eta^k w, k = k + 1
 * The perturbation direction v is g as printed, or g / ||g|| (unit_direction, the
 * normalised reading).  line_search 0 evaluates chi^2 with full products for every
 * trial (literal); line_search 1 uses chi^2(y - beta v) - chi^2(y) =
 * -beta <g, v> + beta^2 Q(v) with Q(v) = sum_PTV w (Dv)^2 + sum_OAR w c^2 (Lv)^2, so a
 * trial is accepted iff beta Q(v) < <g, v>.  That identity needs the OAR term as
 * printed; with the one-sided reading chi^2 is only piecewise quadratic along v and
 * the literal comparison is used whatever line_search says.  The AMS step is the
 * simultaneous form. */
void orc_sa_iteration(const orc_mat *m, const orc_problem *p, const orc_params *q,
                      int64_t *k_io, int64_t *s_io, double *x, orc_iter_info *info) {
  int64_t R = m->R, C = m->C;
  int64_t k = *k_io, s = *s_io;
  double *y = (double *)malloc((size_t)(C ? C : 1) * sizeof(double));
  double *g = (double *)malloc((size_t)(C ? C : 1) * sizeof(double));
  double *yn = (double *)malloc((size_t)(C ? C : 1) * sizeof(double));
  double *dg = (double *)malloc((size_t)(R ? R : 1) * sizeof(double));
  double *lg = (double *)malloc((size_t)(R ? R : 1) * sizeof(double));
  memset(info, 0, sizeof(*info));
  memcpy(y, x, (size_t)C * sizeof(double));
  info->cost_before = orc_cost(m, p, y);
  double cost_y = info->cost_before;
  for (int32_t t = 0; t < q->reductions_n; ++t) {
    orc_gradient(m, p, y, g);
    double G = 0.0;
    for (int64_t j = 0; j < C; ++j) G += g[j] * g[j];
    info->grad_sq = G;
    if (!(G > 0.0)) break;
    /* v (stored in g) and the slope <grad chi^2, v> */
    double slope = G;
    if (q->unit_direction) {
      double nrm = sqrt(G);
      for (int64_t j = 0; j < C; ++j) g[j] = g[j] / nrm;
      slope = nrm;
    }
    const int closed = q->line_search == 1 && p->objective == 0;
    double Q = 0.0;
    if (closed) {
      orc_forward(m, g, dg, lg);
      for (int64_t i = 0; i < R; ++i) {
        if (p->kind[i] & K_OBJ_DOSE) Q += p->w_obj[i] * dg[i] * dg[i];
        if (p->kind[i] & K_OBJ_CDL) Q += p->w_obj[i] * p->c * p->c * lg[i] * lg[i];
      }
      info->q_last = Q;
    }
    int64_t s_start = s;
    int accepted = 0;
    for (;;) {
      s += 1;
      double beta = pow(q->alpha, (double)s);
      info->n_trials++;
      if (beta < BETA_FLOOR) { info->capped = 1; break; }
      if (closed) {
        if (beta * Q < slope) { accepted = 1; info->beta_last = beta; }
      } else {
        for (int64_t j = 0; j < C; ++j) yn[j] = y[j] - beta * g[j];
        double cn = orc_cost(m, p, yn);
        if (cn < cost_y) { accepted = 1; info->beta_last = beta; cost_y = cn; }
      }
      if (accepted) break;
    }
    if (!accepted) { s = s_start; break; }
    for (int64_t j = 0; j < C; ++j) y[j] = y[j] - info->beta_last * g[j];
    info->n_accepted++;
    if (closed) cost_y = orc_cost(m, p, y);
  }
  info->cost_after_perturb = cost_y;
  double ws = pow(q->eta, (double)k);
  info->proximity = orc_ams_simultaneous(m, p, q->lambda, ws, q->normalization, y, x,
                                         &info->n_violated);
  *k_io = k + 1;
  *s_io = s;
  free(y); free(g); free(yn); free(dg); free(lg);
}

/* iter_max outer iterations of orc_sa_iteration (Fig. 3 with a fixed count). */
void orc_solve(const orc_mat *m, const orc_problem *p, const orc_params *q, int64_t iter_max,
               int64_t *k_io, int64_t *s_io, double *x, orc_iter_info *last) {
  for (int64_t it = 0; it < iter_max; ++it) orc_sa_iteration(m, p, q, k_io, s_io, x, last);
}
