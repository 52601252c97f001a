/*
 * fredopt.h - C ABI of the MI355X hot path of superiorized feasibility seeking for
 * simultaneous proton dose and LETd plan optimization (Borys et al., arXiv
 * 2509.20012, Section 2.4.3, Figs. 2-3, Eq. 2).
 *
 * Problem (Section 2.4, Fig. 2): R voxel rows, C pencil-beam columns, sparse
 * influence matrices D (dose per unit fluence, Gy) and L (numerator of the
 * dose-averaged LET of Eq. 1, Gy keV/um per unit fluence; Section 2.2 explains why
 * numerator and denominator are stored separately, and the dose matrix serves as
 * the denominator).  For a fluence x >= 0:
 *     d = D x,   l = L x,   LETd_i = l_i / d_i (0 where d_i = 0),   cDL_i = c l_i
 * with c = 0.04 um/keV (Section 2.4).  Each row carries a bit mask of half-space
 * constraints (Fig. 2) and objective terms (Eq. 2):
 *     FREDOPT_DOSE_LO   d_i >= dose_lo_i              normal a = D_i
 *     FREDOPT_DOSE_HI   d_i <= dose_hi_i              normal a = D_i
 *     FREDOPT_CDL_LO    c l_i >= cdl_lo_i             normal a = c L_i
 *     FREDOPT_CDL_HI    c l_i <= cdl_hi_i             normal a = c L_i
 *     FREDOPT_LETD_HI   LETd_i <= letd_max_i, linearised as l_i - T_i d_i <= 0,
 *                       normal a = L_i - T_i D_i
 *     FREDOPT_OBJ_DOSE  Eq. (2) PTV term   w_obj_i (dose_target_i - d_i)^2
 *     FREDOPT_OBJ_CDL   Eq. (2) OAR term   w_obj_i (cdl_target_i - c l_i)^2
 *
 * Conventions for every call:
 *  - Device pointers everywhere except fredopt_matrices with on_device = 0 and
 *    the host structs (problem, params, state) themselves.  Every array of a
 *    fredopt_problem is a device array of n_rows elements (NULL is accepted when
 *    n_rows = 0).
 *  - The caller owns every buffer it passes.  The library keeps no caller pointer
 *    after a call returns; it reads or writes the caller's arrays only during the
 *    call (work is enqueued on `stream`; the call returns once the stream work that
 *    touches caller buffers is enqueued, except where a call is documented as
 *    synchronising).
 *  - The device workspace is allocated by the caller (size from
 *    fredopt_workspace_bytes) and must stay alive and untouched until
 *    fredopt_free_plan.  The library does not allocate device memory, except a
 *    temporary staging copy of host matrices during fredopt_load_matrices with
 *    on_device = 0 (fredopt_load_matrices_noalloc allocates none).
 *  - `stream` is a hipStream_t (may be the null stream).
 *  - Every call returns FREDOPT_OK or a negative status; on error nothing the
 *    caller owns has been modified and fredopt_last_error() describes the cause,
 *    except FREDOPT_E_NONFINITE raised by an iteration: x then holds the iterate
 *    reached when the non-finite value was detected.  The device checks for NaN or
 *    Inf in every pass of every iteration; once it finds one, every later kernel of
 *    the call skips the plan, so a long solve stops there and the returned state
 *    (k, s) is the one at the detection.
 *  - Calls on one plan must not overlap; calls on distinct plans are independent.
 */
#ifndef FREDOPT_H
#define FREDOPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FREDOPT_OK = 0,
  FREDOPT_E_ARG = -1,        /* null pointer, parameter out of range            */
  FREDOPT_E_SHAPE = -2,      /* inconsistent sizes or row pointers              */
  FREDOPT_E_INDEX = -3,      /* column index out of range or not increasing     */
  FREDOPT_E_NONFINITE = -4,  /* NaN/Inf or negative influence value, or a NaN/Inf
                                produced during an iteration                     */
  FREDOPT_E_WORKSPACE = -5,  /* workspace too small or misaligned               */
  FREDOPT_E_DEVICE = -6,     /* HIP runtime error                               */
  FREDOPT_E_STATE = -7,      /* invalid solver state (k < 0, s < -1)            */
  FREDOPT_E_NOT_IMPLEMENTED = -8
} fredopt_status;

/* Value storage of the influence matrices.  16-bit forms store D_ij / s_j and
 * L_ij / s_j rounded to nearest-even, with one FP32 scale s_j per beamlet (the
 * largest D or L value of column j); products accumulate in FP32.  The _IDX16 forms
 * also keep the column indices of the row-major copy in 16 bits (n_cols <= 65536):
 * 6 bytes per stored entry instead of 12. */
typedef enum {
  FREDOPT_F32 = 0, FREDOPT_F16 = 1, FREDOPT_BF16 = 2, FREDOPT_F16_IDX16 = 3,
  FREDOPT_BF16_IDX16 = 4
} fredopt_dtype;

#define FREDOPT_DOSE_LO 0x01u
#define FREDOPT_DOSE_HI 0x02u
#define FREDOPT_CDL_LO 0x04u
#define FREDOPT_CDL_HI 0x08u
#define FREDOPT_LETD_HI 0x10u
#define FREDOPT_OBJ_DOSE 0x20u
#define FREDOPT_OBJ_CDL 0x40u

/* Normalisation of the simultaneous projection weights (the paper's Fig. 2 is
 * sequential; its text says the projections run in parallel, Section 1):
 * wt_i = weight_scale * w_i / W with W = sum of w over every enabled (row, kind)
 * (CONVEX_ALL, Cimmino weights), over the violated ones (CONVEX_VIOLATED), or 1 (RAW). */
#define FREDOPT_NORM_CONVEX_ALL 0
#define FREDOPT_NORM_CONVEX_VIOLATED 1
#define FREDOPT_NORM_RAW 2

typedef struct fredopt_plan fredopt_plan; /* opaque; created by load, freed by free */

/* Influence matrices in CSR with one sparsity pattern shared by D and L
 * (Section 2.2: an influence matrix per quantity, per pencil beam, sparse).
 *   row_ptr[n_rows + 1]: row_ptr[0] = 0, non-decreasing, row_ptr[n_rows] = nnz
 *   col_idx[nnz]: in [0, n_cols), strictly increasing within a row
 *   d_val[nnz], l_val[nnz]: finite and >= 0
 * storage selects the device value format: FP32, or FP16 / BF16 with one FP32
 * scale per column (scale_j = max over the column of max(D_ij, L_ij)); products
 * always accumulate in FP32. */
typedef struct {
  int64_t n_rows, n_cols, nnz;
  const int64_t *row_ptr;
  const int32_t *col_idx;
  const float *d_val;
  const float *l_val;
  int32_t storage;       /* fredopt_dtype */
  int32_t on_device;     /* 1: the four arrays are device pointers, 0: host pointers */
  int32_t lanes_per_row; /* forward layout: 0 automatic, or 1, 2, 4, 8, 16 lanes per row */
  int32_t gradient_reserve_pct; /* workspace share, in % of the CSC, kept for the
                                   objective-row copy used by the Eq. (2) gradient:
                                   0 = default (25), < 0 = none (the gradient then
                                   streams the full CSC), 1..100 */
} fredopt_matrices;

/* Per-row bounds, priorities and objective data (Fig. 2, its caption, Eq. 2).
 * All arrays are device arrays of n_rows elements; entries whose kind bit is not
 * set are ignored.  w_feas is the AMS priority w_i (> 0), w_obj the Eq. (2) weight
 * (>= 0). */
typedef struct {
  const uint16_t *kind;
  const float *dose_lo, *dose_hi, *cdl_lo, *cdl_hi, *letd_max;
  const float *w_feas, *w_obj, *dose_target, *cdl_target;
  double c; /* um/keV, > 0; 0.04 in the paper (Section 2.4) */
} fredopt_problem;

/* Objective of the perturbations (Eq. 2).  PRINTED: the OAR term
 * w_obj (cdl_target - c l)^2 as the equation prints it (two-sided: it also pulls cDL
 * up towards its target).  ONE_SIDED: the OAR term counts only where
 * c l > cdl_target, so it only pushes cDL down; the cost is then piecewise quadratic
 * along a perturbation and the step search evaluates it on the device for a window
 * of candidate exponents per pass (Fig. 3's trials in order) instead of the closed
 * form.  The PTV term is two-sided in both. */
#define FREDOPT_OBJECTIVE_PRINTED 0
#define FREDOPT_OBJECTIVE_ONE_SIDED 1

/* Parameters of Figs. 2-3: relaxation lambda in (0, 2] (Fig. 2 caption), step base
 * alpha in (0, 1) and weight decay eta in (0, 1] (text after Fig. 3; eta = 1 is
 * accepted for testing), reductions_n >= 0 perturbations per outer iteration
 * (0 = feasibility seeking only), iter_max outer iterations for fredopt_solve.
 * unit_direction 0 perturbs along grad chi^2 as Fig. 3 prints it, 1 along
 * grad chi^2 / ||grad chi^2|| (the step then moves the point by exactly beta). */
typedef struct {
  double lambda, alpha, eta;
  int32_t reductions_n;
  int32_t iter_max;
  int32_t normalization;  /* FREDOPT_NORM_* */
  int32_t objective;      /* FREDOPT_OBJECTIVE_* */
  int32_t unit_direction; /* 0 or 1 */
  int32_t reserved;       /* must be 0 */
} fredopt_params;

/* Solver state of Fig. 3: outer counter k (weights eta^k w) and the global step
 * exponent s (beta = alpha^s, never reset).  A fresh solve starts from k = 0,
 * s = -1.  The remaining fields are outputs of the last outer iteration. */
typedef struct {
  int64_t k, s;
  int64_t n_violated;      /* violated constraints at the AMS input point       */
  double beta;             /* last accepted step alpha^s (0 if none); the point moves
                              by beta times the direction (g, or g / ||g||)      */
  double cost;             /* Eq. (2) at the start of the last outer iteration  */
  double cost_perturbed;   /* Eq. (2) at the perturbed point fed to AMS         */
  double proximity;        /* 1/2 sum (w_i / W_all) v_i^2 / ||a_i||^2 at that point */
  double grad_sq;          /* ||grad chi^2||^2 of the last perturbation         */
  double q;                /* sum w (D g)^2 + sum w c^2 (L g)^2 of that direction */
  int64_t n_active;        /* rows with a non-zero projection coefficient        */
  int32_t projection_path; /* 1: the last sweep used the active-row path, 0: CSC  */
  int32_t reserved;
  int64_t active_entries;  /* stored matrix entries of those rows                 */
} fredopt_state;

/* Bytes of device workspace a plan of this size needs: an upper bound valid for
 * every sparsity pattern with these sizes and the automatic forward layout.
 * Returns 0 for invalid sizes. */
size_t fredopt_workspace_bytes(int64_t n_rows, int64_t n_cols, int64_t nnz, int32_t storage);

/* The exact workspace for one pattern: row_ptr is a HOST array of n_rows + 1
 * offsets; lanes_per_row and gradient_reserve_pct as in fredopt_matrices.  Returns 0
 * for invalid input. */
size_t fredopt_workspace_bytes_csr(int64_t n_rows, int64_t n_cols, const int64_t *row_ptr,
                                   int32_t storage, int32_t lanes_per_row,
                                   int32_t gradient_reserve_pct);

/* Table 2 step (iii): validate the CSR, copy it to the workspace in the device
 * layout (a sliced-ELL copy for the forward products: rows sorted by length inside
 * windows of consecutive rows, lanes_per_row lanes per row, one shared index array
 * and planar D / L values; a CSC copy with rows ascending in every column for the
 * transposed products), compute the per-row FP64 moments sum D^2, sum L^2,
 * sum D L, and return a plan.  `workspace` must be 256-byte aligned device memory
 * of at least fredopt_workspace_bytes_csr(...) bytes.  Synchronises `stream`. */
fredopt_status fredopt_load_matrices(const fredopt_matrices *m, void *workspace,
                                     size_t workspace_bytes, void *stream,
                                     fredopt_plan **out);

/* For callers that cannot allocate device memory (serving loops that admit plans
 * without touching the allocator, harnesses that forbid hipMalloc): the same load
 * and the same plan as fredopt_load_matrices, allocating nothing.  Host-resident
 * matrices (on_device = 0) are staged in a fixed area of the library's own device
 * memory, FREDOPT_NOALLOC_STAGING_BYTES per device, held from the library's load
 * until the process ends; the staged copy needs
 *     align256(8 (n_rows + 1)) + align256(4 nnz) + 2 align256(4 nnz)
 * bytes, and larger host matrices are refused with FREDOPT_E_WORKSPACE (load them
 * from device memory, which needs no staging).  Calls on one device share that
 * area: the library serialises them with a per-device lock inside one process (a
 * call waits while another stages), and the area keeps the last call's contents.
 * The plan's capture stream is created by its first fredopt_solve instead of here.
 * Synchronises `stream`. */
#define FREDOPT_NOALLOC_STAGING_BYTES ((size_t)128 << 20)
fredopt_status fredopt_load_matrices_noalloc(const fredopt_matrices *m, void *workspace,
                                             size_t workspace_bytes, void *stream,
                                             fredopt_plan **out);

/* Releases the host side of a plan (the caller then frees the workspace). */
fredopt_status fredopt_free_plan(fredopt_plan *p);

/* d = D x, LETd = l / d (0 where d = 0) and cDL = c l (Eq. 1, Section 2.4) for a
 * device fluence x[n_cols].  Outputs are device arrays of n_rows floats; any of
 * them may be NULL.  Asynchronous on `stream`. */
fredopt_status fredopt_dose_let(fredopt_plan *p, const float *x, double c, float *dose,
                                float *letd, float *cdl, void *stream);

/* One simultaneous relaxed-projection sweep (the parallel form of Fig. 2) at the
 * device fluence x_inout[n_cols], in place: every violated half-space contributes
 * lambda * wt_i * v_i / ||a_i||^2 * a_i with wt_i = weight_scale * w_i / W, the
 * contributions are summed, and x is clamped to >= 0.  *proximity_out (nullable)
 * receives the proximity of the input point.  Synchronises `stream`. */
fredopt_status fredopt_project_sweep(fredopt_plan *p, const fredopt_problem *pr,
                                     const fredopt_params *q, double weight_scale,
                                     float *x_inout, double *proximity_out, void *stream);

/* One outer iteration k of Fig. 3 from state *st (in/out): reductions_n gradient
 * perturbations of Eq. (2) with beta = alpha^s, s the smallest integer above the
 * previous s for which the cost strictly decreases, then one sweep with weights
 * eta^k w applied to the perturbed point; k += 1.  The gradient only involves rows
 * with objective terms; the plan keeps a copy of their CSC entries, rebuilt when the
 * problem's kind array changes (address or contents).  Synchronises `stream`. */
fredopt_status fredopt_superiorize_step(fredopt_plan *p, const fredopt_problem *pr,
                                        const fredopt_params *q, fredopt_state *st,
                                        float *x_inout, void *stream);

/* q->iter_max outer iterations of fredopt_superiorize_step, captured once as a
 * HIP graph and replayed with all step decisions made on the device.  Resumable:
 * continuing from the returned state reproduces an uninterrupted run bit for bit.
 * Synchronises `stream`. */
fredopt_status fredopt_solve(fredopt_plan *p, const fredopt_problem *pr,
                             const fredopt_params *q, fredopt_state *st, float *x_inout,
                             void *stream);

/* Block-sequential sweep (Fig. 2 takes the constraints one after another on the
 * current fluence; this takes them in consecutive blocks of block_rows rows, in
 * ascending row order): each block is a simultaneous relaxed projection of its own
 * rows' constraints at the current x, with weights weight_scale * w_i / W normalised
 * over that block (q->normalization), and x >= 0 is imposed once after the last
 * block, as Fig. 2 does.  block_rows >= n_rows is the simultaneous sweep of
 * fredopt_project_sweep; otherwise it must be a multiple of 8192 (the layout keeps
 * such blocks of rows contiguous).  Uses the active-row projection for every block.
 * In place on the device fluence x_inout[n_cols].  Synchronises `stream`. */
fredopt_status fredopt_project_sweep_blocks(fredopt_plan *p, const fredopt_problem *pr,
                                            const fredopt_params *q, double weight_scale,
                                            int64_t block_rows, float *x_inout,
                                            void *stream);

/* ---- robustness evaluation ---------------------------------------------------- */

/* Device workspace of fredopt_scenario_dose_let for these n plans (0 for invalid
 * input). */
size_t fredopt_scenario_workspace_bytes(fredopt_plan *const *plans, int32_t n);

/* The robustness evaluation of Section 2.5 (the final plan recomputed under setup
 * and range scenarios; Figs. 4-5 show the spread): dose, LETd and cDL of one device
 * fluence x[n_cols] under n scenario plans, in one launch over all their rows, and
 * per-voxel bands over the scenarios.  plans[i] holds scenario i's matrices; every
 * plan must have the same n_rows (row r is the same voxel in every scenario), n_cols
 * (column j the same beamlet), storage and device, else FREDOPT_E_SHAPE / E_ARG.
 * Outputs are device arrays, any of them NULL: dose, letd, cdl of n * n_rows floats,
 * scenario-major (scenario i's row r at i * n_rows + r); dose_min, dose_max,
 * letd_min, letd_max of n_rows floats (each pair both or neither): the smallest and
 * largest value over the scenarios, exact (no rounding: the values are compared,
 * in any order).  LETd is 0 where a scenario gives the voxel no dose.  `workspace`:
 * 256-byte aligned device memory of fredopt_scenario_workspace_bytes(plans, n)
 * bytes, used only during the call.  Synchronises `stream`. */
fredopt_status fredopt_scenario_dose_let(fredopt_plan *const *plans, int32_t n,
                                         const float *x, double c, float *dose, float *letd,
                                         float *cdl, float *dose_min, float *dose_max,
                                         float *letd_min, float *letd_max, void *workspace,
                                         size_t workspace_bytes, void *stream);

/* ---- evaluation: volume histograms and quantiles ---------------------------------- */

/* Cumulative volume histogram of one region of interest (the DVH, LVH or cDLVH of
 * Figs. 4-5 and Section 2.5): with `values` a device array of n_rows floats (dose,
 * LETd or cDL per voxel row) and `rows` a device array of the region's n row indices,
 * cum[b] (device, n_bins + 1 uint32) = the number of the region's rows whose value is
 * at least b * vmax / n_bins, for b = 0..n_bins (the bin of a value v >= 0 is
 * floor(v * n_bins / vmax) in FP64, values >= vmax fall in bin n_bins; negative and
 * NaN values count in no bin).  Exact integer counts.  1 <= n_bins <= 32768, vmax > 0.
 * Rows outside [0, n_rows) are skipped.  Asynchronous on `stream`. */
fredopt_status fredopt_volume_histogram(const float *values, int64_t n_rows,
                                        const int32_t *rows, int64_t n, double vmax,
                                        int32_t n_bins, uint32_t *cum, void *stream);

/* Nearest-rank quantiles of one region's values, exactly as a sort would give them:
 * out[k] (device, n_q floats) = the value at 1-based rank max(1, ceil(q[k] n)) of the
 * region's values in ascending order, for host q[k] in (0, 1], 1 <= n_q <= 16.  D95
 * of a PTV is q = 0.05 of its doses (the dose the hottest 95 % receive at least), D98
 * q = 0.02; the cDL30 of an OAR that sets its percentile constraint from a forward
 * calculation (Section 2.4.1) is q = 0.70 of its cDL.  An empty region gives 0.
 * Rows as for fredopt_volume_histogram.  Asynchronous on `stream`. */
fredopt_status fredopt_roi_quantiles(const float *values, int64_t n_rows, const int32_t *rows,
                                     int64_t n, const double *q, int32_t n_q, float *out,
                                     void *stream);

/* Thread-local description of the last failing call on this thread. */
const char *fredopt_last_error(void);

/* ---- introspection and measurement ------------------------------------------ */

typedef struct {
  int64_t n_rows, n_cols, nnz;
  int64_t sell_slots, csc_slots;  /* stored entries including padding               */
  int64_t bytes_per_sell_slot, bytes_per_csc_slot;
  int64_t n_slices, tr_items, row_items;
  int64_t workspace_bytes;
  int64_t grad_entries;     /* entries the gradient pass streams (after a problem was
                               prepared: objective rows only, or nnz), else 0     */
  int64_t obj_entries;      /* entries of the objective-row forward view (0 if unused) */
  int32_t storage, lanes_per_row, fwd_grid, tr_chunk;
  int32_t lds_x;    /* 1 if the forward kernels stage the vector in LDS */
  int32_t schedule; /* 1: objective-row view in use (one all-row forward product per
                       outer iteration), 0: two all-row forward products */
  int32_t scatter_wgs;      /* workgroups of the active-row projection (0: off)  */
  int64_t scatter_max_rows; /* largest active-row count that takes that path     */
  int32_t obj_lanes_per_row; /* lanes per row of the objective-row view (0: unused) */
  int32_t fwd_schedule;      /* all-row forward: 1 groups from a counter, 2 round robin */
  int32_t scatter_lanes;     /* lanes of the active-row scatter per row (4..64)  */
  int64_t row_copy_slots;    /* slots of its row-contiguous copy (rows padded to 4) */
} fredopt_plan_info;

fredopt_status fredopt_get_plan_info(const fredopt_plan *p, fredopt_plan_info *info);

/* Kernel identifiers of one outer iteration. */
#define FREDOPT_KERNEL_FWD_OBJ 0   /* d, l and Eq. (2) coefficients at x            */
#define FREDOPT_KERNEL_TR_GRAD 1   /* gradient chunks of the transposed product     */
#define FREDOPT_KERNEL_FWD_DIR 2   /* D g, L g and the Q partials                   */
#define FREDOPT_KERNEL_ROWS 3      /* move d, l; constraint residuals               */
#define FREDOPT_KERNEL_TR_PROJ 4   /* projection chunks of the transposed product   */
#define FREDOPT_KERNEL_FWD_RESID 5 /* d, l and residuals (reductions_n = 0)         */
#define FREDOPT_KERNEL_COL 6       /* per-column sums: gradient or update and clamp */
#define FREDOPT_KERNEL_FINALIZE 7  /* plan scalars: step decision, weights          */
#define FREDOPT_KERNEL_ACTIVE_LIST 8 /* list of rows with a projection coefficient  */
#define FREDOPT_KERNEL_SCATTER 9   /* transposed product over those rows only       */
#define FREDOPT_KERNEL_SCATTER_SUM 10 /* its per-workgroup sums; projection update  */
#define FREDOPT_KERNEL_LINE_SEARCH 11 /* step search of the one-sided objective   */
#define FREDOPT_NUM_KERNELS 12

/* Runs n_iters outer iterations (as fredopt_superiorize_step would) launching each
 * kernel separately with HIP events around it on `stream`, and writes the mean
 * duration in milliseconds of every kernel id to ms_out[FREDOPT_NUM_KERNELS]
 * (0 for kernels not launched) and the launch count to count_out (nullable).
 * Advances *st and x like the same number of steps.  Synchronises `stream`. */
fredopt_status fredopt_profile_kernels(fredopt_plan *p, const fredopt_problem *pr,
                                       const fredopt_params *q, fredopt_state *st,
                                       float *x_inout, int32_t n_iters, void *stream,
                                       double *ms_out, int64_t *count_out);

/* Autotuner: times the candidate workgroups-per-CU counts of the forward kernel and
 * chunk sizes of the transposed kernel on this plan (its own matrices, fluence x)
 * and keeps the fastest.  Synchronises `stream`. */
fredopt_status fredopt_autotune(fredopt_plan *p, const float *x, void *stream);

/* Sets the forward workgroups per CU (1..8, capped by LDS), the transposed chunk
 * size (slots per work item, a multiple of 256) and how the all-row forward pass
 * hands out its slice groups (1: from a counter, 2: round robin); 0 keeps the
 * current value. */
fredopt_status fredopt_set_tuning(fredopt_plan *p, int32_t fwd_wgs_per_cu, int32_t tr_chunk,
                                  int32_t fwd_schedule);

/* The projection of Fig. 2 needs D^T and L^T applied to the rows' coefficients, which
 * are zero for every satisfied constraint.  When at most max_active_rows rows have a
 * non-zero coefficient, the plan applies the transposes to those rows only (read
 * through the forward layout, summed in 64-bit fixed point, order independent);
 * otherwise it streams the column-major copy.  The choice is made on the device at
 * every sweep.  Both paths give the same result up to FP32 rounding of the sums.
 * n_workgroups: 0 default (one per 64k stored entries, at most one per compute
 * unit), -1 disables the active-row path, 1..256 sets the count.  max_active_rows:
 * -1 default (a quarter of the rows).  The column sums live in LDS (8 * n_cols bytes
 * per workgroup) when they fit, otherwise in the workspace, added with device-scope
 * integer atomics (still order independent). */
fredopt_status fredopt_set_scatter(fredopt_plan *p, int32_t n_workgroups,
                                   int64_t max_active_rows);

/* ---- batches: many plans iterated by the same launches ------------------------
 *
 * Fig. 3 run for several independent plans (patients, or robustness scenarios of
 * one patient, each with its own matrices and problem) by one sequence of kernel
 * launches: each launch takes the work items of every plan, each outer iteration is
 * one hipGraph replay.  A plan's arithmetic is the one it has alone (its schedule,
 * its work items; the active-row projection gets workgroups in proportion to the
 * plan, which its exact integer sums do not see), so its iterates are the same bit
 * for bit.  Plans keep their own workspaces and states; the batch only adds a table
 * of descriptors and the concatenated work lists. */
typedef struct fredopt_batch fredopt_batch;

/* Device bytes of the batch workspace for these plans (0 on a NULL plan). */
size_t fredopt_batch_workspace_bytes(fredopt_plan *const *plans, int32_t n);

/* Binds plans[i] to problems[i] (checked and prepared as by fredopt_solve) and
 * builds the batch in the caller's workspace (device memory, at least
 * fredopt_batch_workspace_bytes, owned by the caller, kept until
 * fredopt_batch_free).  All plans need the same storage and device; a plan may
 * belong to one batch at a time and must not be used on its own meanwhile.  The
 * problem structs are copied; the device arrays they point to must stay valid
 * while the batch lives.  Synchronises `stream`. */
fredopt_status fredopt_batch_create(fredopt_plan *const *plans, int32_t n,
                                    const fredopt_problem *problems, void *workspace,
                                    size_t workspace_bytes, void *stream,
                                    fredopt_batch **out);

/* n_iters outer iterations of every plan of the batch, plan i from states[i] and
 * the device fluence x[i] (in place); the states are updated as by fredopt_solve.
 * Synchronises `stream`. */
fredopt_status fredopt_batch_solve(fredopt_batch *b, const fredopt_params *q,
                                   fredopt_state *states, float *const *x, int32_t n_iters,
                                   void *stream);

fredopt_status fredopt_batch_free(fredopt_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* FREDOPT_H */
