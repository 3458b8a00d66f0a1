/*
 * elses.h -- C ABI of the MI355X (gfx950) generalized shifted Krylov solver.
 *
 * The library solves the generalized shifted linear equations
 *
 *     (z_k B - A) x_{j,k} = e_j ,   k = 1..K,  Im z_k > 0,
 *
 * for many basis columns j of a sparse real-symmetric Hamiltonian A and a
 * sparse real-symmetric positive-definite overlap B (paper Sec. III-A,
 * Eqs. 9 and 13).  All shifts of one column share one Krylov subspace
 * (Sec. III-B, Eq. 14).  The solutions feed the energy integral for the
 * density matrix (Eq. 12) and the projected quantities e_j^T rho X e_j
 * (Eq. 7), which only need rho on the sparsity pattern of X (Sec. II-B,
 * nearsightedness).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are given per atom block (Sec. II-C: composite index
 *   i <-> (I, alpha)).  Atoms carry 4 orbitals (C: s, px, py, pz) or 1 (H: s),
 *   in any order; orbitals are numbered atom by atom.  Numbering atoms with
 *   spatial locality (e.g. along a space-filling curve) makes the sparse
 *   products cache-friendly; it does not change results.
 * - "Host" pointers are read during the call only; the caller keeps
 *   ownership.  "Device" pointers are GPU memory the caller allocated (for
 *   example torch tensors); the library never frees or retains them.
 * - Work is enqueued on the context's HIP stream.  Entry points that return
 *   results synchronise that stream before returning.
 * - Complex numbers are two doubles (re, im) interleaved.
 * - No exceptions cross the ABI.  A non-OK status leaves a message for
 *   elses_last_error().  Argument errors are reported before any launch.
 */
#ifndef ELSES_H
#define ELSES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ELSES_OK = 0,
    ELSES_ERR_INVALID_ARG = 1,    /* bad argument; nothing was launched          */
    ELSES_ERR_HIP = 2,            /* a HIP runtime call failed                    */
    ELSES_ERR_OOM = 3,            /* device allocation failed                     */
    ELSES_ERR_NOT_SPD = 4,        /* overlap B is not positive definite           */
    ELSES_WARN_NOT_CONVERGED = 5  /* outputs written; some (j,k) missed the tol   */
} elses_status;

enum { ELSES_FP64 = 0, ELSES_MIXED = 1 };          /* storage precision of A, B  */
enum { ELSES_OUT_PATTERN = 0, ELSES_OUT_FULL = 1 }; /* extent of x_out            */

typedef struct elses_ctx_s *elses_ctx;
typedef struct elses_mat_s *elses_mat;

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *out receives the handle. */
elses_status elses_ctx_create(int device, void *hip_stream, elses_ctx *out);
void elses_ctx_destroy(elses_ctx ctx);
/* Message of the last failed call on this context (static storage of the
 * context, valid until the next call). Never NULL. */
const char *elses_last_error(elses_ctx ctx);

/*
 * System description (all HOST pointers, copied by elses_mat_create).
 *  n_atoms        number of atoms N
 *  n_orb[N]       orbitals per atom: 4 or 1
 *  blk_row_ptr    [N+1] block-row pointer; row I lists its coupled atoms J,
 *                 including I itself, in ascending J; the block pattern must
 *                 be symmetric ((I,J) present <=> (J,I) present)
 *  blk_col        [nnzb] atom index J of each block
 *  A_val, B_val   values of each block (n_orb[I] x n_orb[J], row-major),
 *                 blocks concatenated in pattern order; A and B share the
 *                 pattern; both must be symmetric (paper Sec. II-A)
 *  pos            [3N] atom positions (Angstrom); may be NULL when no region
 *                 solves are requested
 *  box            side of the periodic cube (Angstrom); <= 0: not periodic
 */
typedef struct {
    int32_t n_atoms;
    const int8_t *n_orb;
    const int64_t *blk_row_ptr;
    const int32_t *blk_col;
    const double *A_val;
    const double *B_val;
    const double *pos;
    double box;
} elses_system;

/*
 * Upload a system and prepare it for solves.  precision: ELSES_FP64 keeps A
 * and B in FP64; ELSES_MIXED additionally stores FP32 planes used by the
 * overlap solve with FP64 residual refinement.  Estimates the spectral
 * interval of B (used by the overlap solve) and fails with ELSES_ERR_NOT_SPD
 * if B is not positive definite.
 */
elses_status elses_mat_create(elses_ctx ctx, const elses_system *sys, int precision, elses_mat *out);
void elses_mat_destroy(elses_mat mat);

/* Number of orbitals M, and the largest pattern length max_j |P_j|. */
elses_status elses_mat_info(elses_mat mat, int64_t *M, int64_t *pmax, double *b_lo, double *b_hi);

/*
 * Pattern layout.  For column j on atom J, P_j is the ascending list of
 * orbitals of the atoms coupled to J (the rows i with B_ij structurally
 * present; Sec. II-B: rho_ij is needed only where X_ij != 0).
 * pat_off (HOST, n_cols+1) receives the prefix sums of |P_j| over `cols`;
 * rows (HOST, may be NULL) receives the concatenated row lists.
 */
elses_status elses_pattern(elses_mat mat, int32_t n_cols, const int32_t *cols, int64_t *pat_off, int32_t *rows);

typedef struct {
    double tol;          /* relative residual ||e_j - (z B - A) x|| per (j,k); default 1e-8 */
    int32_t max_outer;   /* outer (Lanczos) iterations per column; default 20000            */
    double inner_tol;    /* relative residual of each overlap solve; default 1e-13          */
    int32_t out_mode;    /* ELSES_OUT_PATTERN or ELSES_OUT_FULL (not on region tiles)       */
    int32_t slots;       /* columns advanced together (multiple of 64); 0 = autotune        */
    int32_t use_mixed;   /* 1: FP32 overlap solve + FP64 refinement (needs ELSES_MIXED)     */
    int32_t audit;       /* 1: recompute FP64 true residuals (ELSES_OUT_FULL only)          */
    int32_t variant;     /* sparse passes: 0 auto, 1 direct gathers, 2 / 3 LDS-staged       */
                         /* gathers (8- / 4-atom clusters), 4 row groups sharing gathers   */
    int32_t graph;       /* 1: capture the outer iterations in a HIP graph and replay it    */
                         /* on a private stream (pass timing is not sampled); default 0.    */
                         /* No effect on compact region sets (already one launch).          */
    int32_t audit_every; /* compact region sets, pattern mode: the columns c with           */
                         /* c % audit_every == 0 are also carried on every row of their     */
                         /* region and their resid_out entries receive the recomputed FP64  */
                         /* true residual instead of the estimate; 0 (default) = none       */
    int32_t precond;     /* 1 = overlap solves preconditioned with the learned M of          */
                         /* elses_mat_set_preconditioner; default 0.  Compact region sets   */
                         /* (created after it): conjugate gradients with M; a region whose  */
                         /* M fails (a non-positive curvature, or inner_max steps without   */
                         /* reaching inner_tol) falls back to the plain iteration.  Global  */
                         /* solves (FP64 only, no graph): Richardson steps                  */
                         /* x <- x + tau_k M (s - B x) with the Chebyshev roots of M B's    */
                         /* interval; a matrix whose M is not SPD runs the plain steps      */
                         /* (one fallback counted).  Tile region sets: INVALID_ARG.         */
    int32_t inner_max;   /* preconditioned CG steps per solve before the fallback; 200      */
} elses_opts;

/* Fill *o with the defaults listed above. */
void elses_opts_default(elses_opts *o);

/*
 * Solve (z_k B - A) x = e_j for every j in cols (HOST, n_cols distinct
 * column indices in [0, M)) and every shift (HOST, n_shifts complex, Im > 0).
 *
 * x_out (DEVICE, complex interleaved), may be NULL:
 *   ELSES_OUT_PATTERN: column c occupies [pat_off[c]*K, pat_off[c+1]*K)
 *                      complex entries laid out [K][|P_j|];
 *   ELSES_OUT_FULL:    [n_cols][K][M].
 * iters_out (DEVICE int32 [n_cols]) outer iterations, may be NULL.
 * resid_out (DEVICE double [n_cols*K]) residual per (j,k): the recursive
 *   estimate, or with opts->audit the recomputed FP64 true residual; may be
 *   NULL.  Mixed solves (use_mixed) solve the pencil of the FP32-rounded A
 *   and B: their audit recomputes the residual of that pencil in FP64.
 * Returns ELSES_WARN_NOT_CONVERGED if some (j,k) ended above tol (outputs
 * are still written).
 */
elses_status elses_shifted_solve(elses_ctx ctx, elses_mat mat, int32_t n_cols, const int32_t *cols,
                                 int32_t n_shifts, const double *shifts, const elses_opts *opts,
                                 double *x_out, int32_t *iters_out, double *resid_out);

/*
 * Density-matrix elements on the pattern (Eq. 12 discretised on the shifts):
 *     rho_ij = sum_k Im(c_k x_{j,k,i}),  i in P_j,
 * with complex weights c (HOST, n_shifts complex; for the Fermi-weighted
 * midpoint rule c_k = -(1/pi) w_k f(Re z_k)).
 * rho_out (DEVICE double, pattern layout pat_off) receives rho.
 * traces_out (HOST double[2]) receives sum_j e_j^T rho B e_j and
 * sum_j e_j^T rho A e_j over the requested columns (Eq. 7), may be NULL.
 * col_traces_out (DEVICE double [n_cols][2]) per-column values, may be NULL.
 * x_out / iters_out / resid_out as in elses_shifted_solve (may be NULL).
 */
elses_status elses_density_matrix(elses_ctx ctx, elses_mat mat, int32_t n_cols, const int32_t *cols,
                                  int32_t n_shifts, const double *shifts, const double *c,
                                  const elses_opts *opts, double *rho_out, double *traces_out,
                                  double *col_traces_out, double *x_out, int32_t *iters_out,
                                  double *resid_out);

/*
 * Kernel timing of the overlap-solve pass (diagnostics for roofline reports).
 * When enabled, solves time the back-to-back Richardson steps 2 .. d-2 of
 * the overlap solve (FP32 in mixed solves) every `stride`-th outer
 * iteration with one pair of HIP events on the context stream (stride >= 1;
 * 0 disables).  The counters accumulate over calls until reset by a new
 * stride.
 *   launches       passes timed
 *   avg_us         mean duration of a timed pass (microseconds)
 *   bytes          algorithmic HBM bytes of one pass: B's values (8 or 4
 *                  bytes each) and index arrays once, plus three [M][slots]
 *                  blocks (the gathered iterate, the right-hand side, the new
 *                  iterate; 8 or 4 bytes per entry)
 *   flops          2 * nnz * slots + 3 * M * slots
 *   total_passes   all passes (A and B products) launched by solves
 * Region solves in the compact layout time their launches instead: the
 * launches of the width groups (4, 2 or 1 columns per region) overlap, and
 * one solve counts as one launch from the first group's start to the last
 * group's end; bytes and flops are the means over the timed solves of the
 * algorithmic traffic of all groups: per outer step of each region its sparse
 * products (the A product, the Richardson steps of the region's own plan and,
 * in mixed precision, the refinement product; a 2-byte index plus the value,
 * 4 or 8 bytes, per nonzero, or for Richardson steps on the half layout of B
 * 6 bytes per stored off-diagonal pair plus 4 per diagonal entry), the
 * carried x and p (read and written, 64 bytes
 * per shift and row) and its Lanczos vectors in scratch (18 x 8 bytes per
 * row and column); slots = the column width of the group that moved most
 * bytes.  A compact launch holds at most one workgroup (one region) per CU.
 * Multiple Arnoldi calls (elses_arnoldi, elses_regions_arnoldi) sample their
 * Gram-Schmidt update passes instead (every stride-th launch, one launch per
 * sample; block b subtracts the projections of two candidates on the 2b basis
 * vectors so far): bytes = the mean over samples of 2b basis blocks and two
 * candidate blocks read, two candidate blocks written, the coefficients read
 * and the partial Gram entries written; flops = 2 (4b [+ 3]) per row and
 * lane; slots = lanes (segments x lane width).
 */
elses_status elses_ctx_set_profiling(elses_ctx ctx, int32_t stride);
elses_status elses_ctx_pass_stats(elses_ctx ctx, int64_t *launches, double *avg_us, double *bytes, double *flops,
                                  int64_t *total_passes, int32_t *slots);
/* Load balance of the profiled compact region solves since the last
 * elses_ctx_set_profiling: the mean over those solves of the share of
 * resident workgroup time spent without a region in the vector-width group
 * that moves most bytes, 1 - (sum of its workgroup lifetimes) / (its
 * workgroups x span of the solve), from per-workgroup stamps
 * of the device's constant-rate clock (the analogue of the paper's barrier
 * time from load imbalance, Table II); solves = how many were measured. */
elses_status elses_ctx_region_idle(elses_ctx ctx, double *idle_share, int64_t *solves);

/*
 * Time `reps` back-to-back launches of one sparse pass on scratch blocks of
 * `slots` right-hand sides (a multiple of 64) with pass kernels `variant`
 * (as in elses_opts).  kind: 0 the A pass of a Lanczos step, 1 a
 * Richardson step of the overlap solve, 2 the last step (with the dot
 * products of the Lanczos step), 3 the plain product, 9 the first step
 * (forming its operand from two vectors); mixed precision (matrix created
 * with ELSES_MIXED): 4 the A pass, 5 an FP32 Richardson step, 6 the FP64
 * residual refinement, 7 the last FP32 step, 8 the plain FP32 product,
 * 10 the first FP32 step.  *avg_us receives the mean launch time
 * measured with HIP events on the context stream.  Used by the slot and
 * variant autotuner and by performance diagnostics.
 */
elses_status elses_time_pass(elses_ctx ctx, elses_mat mat, int32_t kind, int32_t variant, int32_t slots,
                             int32_t reps, double *avg_us);

/*
 * Observables from stored solutions (no new solves).
 *
 * Pattern blocks: the pattern P_j of a column j lists, for each atom I
 * coupled to j's atom (ascending), the orbitals of I.  blk_off (HOST
 * [n_cols+1]) receives the prefix sums of the number of coupled atoms over
 * `cols`, blk_atom (HOST, may be NULL) the atom I of each block.
 */
elses_status elses_pattern_blocks(elses_mat mat, int32_t n_cols, const int32_t *cols, int64_t *blk_off,
                                  int32_t *blk_atom);
/*
 * Density matrix on the pattern for new weights c (HOST complex [n_shifts])
 * from solutions x (DEVICE, pattern layout of elses_shifted_solve for the
 * same cols and shifts): rho_ij = sum_k Im(c_k x_{j,k,i}) (Eq. 12 on the
 * shifts).  rho_out (DEVICE, pattern layout), col_traces_out (DEVICE
 * [n_cols][2]: e_j^T rho B e_j, e_j^T rho A e_j, Eq. 7) and traces_out (HOST
 * [2], their sums) may be NULL.  icohp_out (DEVICE double [blk_off[n_cols]],
 * may be NULL) receives for every column j and coupled atom I the sum over
 * I's orbitals alpha of rho_{(I,alpha), j} A_{j, (I,alpha)}: summed over the
 * orbitals of j's atom J this is the connectivity (ICOHP) C_IJ of the
 * paper's network analysis (Sec. V-A), whose total over all atom pairs is
 * the energy Tr[rho A] (Eq. 4).
 */
elses_status elses_density_reweight(elses_ctx ctx, elses_mat mat, int32_t n_cols, const int32_t *cols,
                                    int32_t n_shifts, const double *c, const double *x, double *rho_out,
                                    double *traces_out, double *col_traces_out, double *icohp_out);
/*
 * Chemical potential (Eq. 3): with the Fermi-weighted midpoint rule
 * c_k = -(1/pi) w_k f(Re z_k; mu, tau) (w HOST [n_shifts] quadrature
 * widths), bisect mu in [mu_lo, mu_hi] until the interval is below mu_tol so
 * that sum_j e_j^T rho B e_j over cols equals `target`, re-weighting the
 * stored solutions x (DEVICE, pattern layout).  mu_out / count_out (HOST)
 * receive mu and the count there.  The target must lie between the counts
 * at mu_lo and mu_hi.
 */
elses_status elses_chemical_potential(elses_ctx ctx, elses_mat mat, int32_t n_cols, const int32_t *cols,
                                      int32_t n_shifts, const double *shifts, const double *w, const double *x,
                                      double tau, double target, double mu_lo, double mu_hi, double mu_tol,
                                      double *mu_out, double *count_out);

/*
 * Autotuner of the sparse passes.  Times one Richardson step (FP64, or FP32
 * with mixed != 0) for the grouped passes (4, 2 or 1 waves per row group x
 * XCD placements 0, 1, 3) and the direct passes at 256 .. 2048 slots (at most
 * max_slots; 0 = 2048), and keeps the configuration with the lowest time
 * per column in the matrix: later solves with opts.variant == 0 and
 * opts.slots == 0 use it (slots capped by the column count).  Outputs (HOST,
 * may be NULL): the chosen variant code (as opts.variant, placement in bits
 * 4-5), slot count and time per column and pass in nanoseconds.
 */
elses_status elses_autotune(elses_ctx ctx, elses_mat mat, int32_t mixed, int32_t max_slots, int32_t *variant_out,
                            int32_t *slots_out, double *ns_per_column_out);

/* Sparse products with the uploaded matrices (diagnostics and tests):
 * y = X x for X = A (which=0) or B (which=1); x, y DEVICE double [M][nvec]
 * (row-major, nvec contiguous).  For nvec a multiple of 64 the pass kernels
 * of `variant` (as in elses_opts) run; any other nvec uses a generic
 * one-thread-per-entry kernel. */
elses_status elses_spmm(elses_ctx ctx, elses_mat mat, int which, int32_t variant, int32_t nvec, const double *x,
                        double *y);

/*
 * Region problems (paper Sec. III-B: the real-space projection solves each
 * column's equations on the principal sub-pencil (A_r, B_r) of the atoms
 * within a radius of the column's atom; Eq. 7 needs only the column's own
 * pattern).  A region set is built once and then solved for any shifts.
 *
 * elses_regions_create: region r is centred on atom centres[r] (HOST, n_regions
 * distinct atoms) with radius radii[r] (HOST, Angstrom, > 0); it holds the atoms
 * whose minimum-image distance to the centre is <= radius (the matrix needs
 * pos, and box for periodic images).  Its columns are the orbitals of the
 * centre atom, region by region in the order given.
 *
 * Layouts (tile_width):
 *  0        compact (default): every region keeps its own sub-pencil (at most
 *           8192 orbitals per region, and its overlap iterate must fit in LDS);
 *           one persistent launch per column-width group solves them, one
 *           workgroup per region at a time and at most one per CU, taking
 *           regions from a device queue costliest first (nonzeros x sqrt(kappa
 *           of the region's B)), with every step of a
 *           region's solve (outer Lanczos steps, overlap solves with the
 *           Chebyshev-Richardson plan of the region's own overlap interval,
 *           shift updates, density assembly) inside the launch; in mixed
 *           precision the FP32 Richardson steps of regions with 1 or 2
 *           columns read B's symmetric pairs once (a half layout built
 *           with the set), summing the transpose half as 32-bit fixed
 *           point, so results stay reproducible run to run;
 *  64, 128  tiles: consecutive regions (which should be spatial neighbours)
 *           are packed into tiles of tile_width column slots of one
 *           block-diagonal matrix that advance through one launch sequence
 *           per outer step (the layout multiple Arnoldi needs).
 * The set keeps its data on the device until destroyed, and depends on
 * `mat`, which must outlive it.
 */
typedef struct elses_regions_s *elses_regions;
elses_status elses_regions_create(elses_ctx ctx, elses_mat mat, int32_t n_regions, const int32_t *centres,
                                  const double *radii, int32_t tile_width, elses_regions *out);
/* As elses_regions_create, with orb_mask (HOST uint8 [n_regions], may be
 * NULL) selecting the centre's orbitals that are solved as columns: bit q set
 * = orbital q of the centre atom (0 = all orbitals).  Columns sampled on the
 * same atom thus share one region (one solve). */
elses_status elses_regions_create_ex(elses_ctx ctx, elses_mat mat, int32_t n_regions, const int32_t *centres,
                                     const double *radii, const uint8_t *orb_mask, int32_t tile_width,
                                     elses_regions *out);
void elses_regions_destroy(elses_regions reg);
/* Sizes and layout of a region set (HOST outputs, each may be NULL):
 * n_cols columns; n_tiles tiles (0 for the compact layout); rows_total rows of
 * all tiles' atom unions (compact: sum over regions of the padded row count
 * times the region's vector width, so that useful_rows / rows_total is the
 * share of useful lane-rows, as useful_rows / (rows_total x tile_width) is in
 * the tile layout); useful_rows = sum over columns of their region's orbital
 * count;
 * cols [n_cols] global orbital of each column; pat_off [n_cols+1] offsets of
 * each column's pattern P_j in the caller's matrix (as elses_pattern);
 * region_orbitals [n_regions] orbitals of each region. */
elses_status elses_regions_info(elses_regions reg, int32_t *n_cols, int32_t *n_tiles, int64_t *rows_total,
                                int64_t *useful_rows, int32_t *cols, int64_t *pat_off, int32_t *region_orbitals);
/* Region of each column (HOST int32 [n_cols], in the column order of
 * elses_regions_info). */
elses_status elses_regions_columns(elses_regions reg, int32_t *col_region);
/* Overlap interval of each region of a compact set (HOST double [n_regions]
 * each): the extreme Ritz values of the region's B from 40 Lanczos steps at
 * creation, widened by 2 % of the width and 1e-3 relative on each side and
 * kept inside B's interval (a region's B is a principal submatrix of B:
 * its spectrum lies inside B's, Cauchy interlacing).  Each region's overlap
 * solves take the Chebyshev-Richardson plan of its own interval.  Tile sets:
 * ELSES_ERR_INVALID_ARG. */
elses_status elses_regions_overlap_intervals(elses_regions reg, double *lo, double *hi);
/* Solve (z_k B_r - A_r) x = e_j for every column of every region and every
 * shift (HOST, Im z > 0), in pattern mode: x_out, rho_out, col_traces_out,
 * iters_out and resid_out are laid out as in elses_density_matrix for the
 * column list of elses_regions_info (pattern rows outside the region hold 0).
 * c (HOST complex weights) may be NULL when no density output is requested.
 * opts: as elses_opts; use_mixed needs a matrix created with ELSES_MIXED.
 * Tile layout: out_mode must be ELSES_OUT_PATTERN, variant 0 or a grouped
 * variant.  Compact layout: variant and slots are ignored; ELSES_OUT_FULL
 * writes, per column in order, a [K][m_r] block of its region's vectors in
 * the region's orbital order (atoms ascending; m_r = region_orbitals), and
 * with opts->audit resid_out receives the FP64 true residuals
 * ||e_j - (z_k B_r - A_r) x||_2 of the pencil solved (the FP32-rounded one
 * for use_mixed); opts->audit_every audits a subset in pattern mode. */
elses_status elses_regions_solve(elses_ctx ctx, elses_regions reg, int32_t n_shifts, const double *shifts,
                                 const double *c, const elses_opts *opts, double *x_out, double *rho_out,
                                 double *traces_out, double *col_traces_out, int32_t *iters_out,
                                 double *resid_out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * solve as elses_regions_solve on a compact region set, with every work
 * buffer taken from a fixed scratch array that the library holds on each GPU
 * (256 MiB per GPU, for the life of the process).  It calls no hipMalloc or
 * hipFree and creates no stream or event; the column-width groups run one
 * after another on the context stream, with as many workgroups as the
 * scratch holds.  Outputs, arguments and results are those of
 * elses_regions_solve (profiling statistics are not sampled).  A solve whose
 * per-column state does not fit (about K x pattern length x 32 bytes per
 * column plus K x 76 bytes, with K the shift count) returns
 * ELSES_ERR_INVALID_ARG with the size it needs.  Every call on a GPU shares
 * that GPU's array and leaves its contents behind: calls that overlap on one
 * GPU (from several threads or streams) race, and must be serialised by the
 * caller.  Tile region sets return ELSES_ERR_INVALID_ARG.
 */
elses_status elses_regions_solve_noalloc(elses_ctx ctx, elses_regions reg, int32_t n_shifts, const double *shifts,
                                        const double *c, const elses_opts *opts, double *x_out, double *rho_out,
                                        double *traces_out, double *col_traces_out, int32_t *iters_out,
                                        double *resid_out);

/*
 * Learned block sparse approximate inverse (SPAI) of the overlap B.
 *
 * The overlap solves B v = s of the method (paper Sec. III-B: B^{-1} enters
 * every step of the generalized problem) can be preconditioned by an
 * approximate inverse M on B's own block pattern.  A multilayer perceptron
 * predicts the blocks M_IJ of the upper pairs I <= J (M_JI = M_IJ^T) from
 * per-pair features; it is trained on the exact blocks of B^{-1}, which the
 * overlap solve itself computes for small systems.
 *
 * Pairs: the upper pairs (I <= J) of the block pattern, atom row by atom
 * row, ascending J.  Features (FP32 [n_pairs][40]): displacement r_J - r_I
 * over 4 A (3), its length over 4 A, 4-orbital flags of I and J, 10 B_IJ
 * zero-padded to 4 x 4 (16), 10 (E^2)_IJ with E = B - I zero-padded (16),
 * 1 if I == J, 0.  Network: 40 -> 128 -> 128 -> 128 -> 16, exact GELU after
 * the hidden layers, output the 4 x 4 block (valid part n_I x n_J).
 * Parameters: ELSES_MLP_PARAMS FP32 values W1[128][40] b1[128] W2[128][128]
 * b2[128] W3[128][128] b3[128] W4[16][128] b4[16] (DEVICE, caller-owned).
 * Targets (FP32 [n_pairs][16]) with their valid-entry mask (1 / 0).
 * Loss: sum over valid entries of (output - target)^2 / number of valid
 * entries.
 */
#define ELSES_MLP_PARAMS 40336
/* Number of upper pairs; pairs (HOST int32 [n][2], may be NULL) receives (I, J). */
elses_status elses_spai_pairs(elses_mat mat, int64_t *n_pairs, int32_t *pairs);
/* feat (DEVICE float [n_pairs][40]); needs atom positions. */
elses_status elses_spai_features(elses_ctx ctx, elses_mat mat, float *feat);
/* Exact blocks (B^{-1})_IJ from overlap solves of all unit vectors (to
 * 1e-13), target and mask (DEVICE float [n_pairs][16]); for M <= 65536. */
elses_status elses_spai_targets(elses_ctx ctx, elses_mat mat, float *target, float *mask);
/* Loss (HOST) and its gradient (DEVICE float [ELSES_MLP_PARAMS]) over n rows
 * of features / targets / masks (DEVICE), FP32 forward and backward passes. */
elses_status elses_mlp_loss_grad(elses_ctx ctx, const float *params, int64_t n, const float *feat,
                                 const float *target, const float *mask, double *loss, float *grad);
/* `steps` Adam steps (lr, beta 0.9 / 0.999, eps 1e-8) on mini-batches of
 * `batch` rows drawn by seeded shuffles; params (DEVICE) updated in place;
 * loss_history (HOST double [steps], may be NULL) receives each batch loss. */
elses_status elses_spai_train(elses_ctx ctx, float *params, int64_t n, const float *feat, const float *target,
                              const float *mask, int32_t steps, int32_t batch, double lr, uint64_t seed,
                              double *loss_history);
/* Network outputs (DEVICE float [n][16]) for n feature rows; bf16 != 0: BF16
 * weights and activations (round to nearest even) on the matrix cores with
 * FP32 accumulation and FP32 biases (feat must then be 16-byte aligned, else
 * ELSES_ERR_INVALID_ARG); otherwise FP32 throughout. */
elses_status elses_spai_predict(elses_ctx ctx, const float *params, int64_t n, const float *feat, int32_t bf16,
                                float *out);
/* M on B's pattern: features, inference and assembly (diagonal blocks
 * symmetrised).  M_vals (DEVICE double, as many values as B) is in the
 * library's internal block order: an opaque buffer for elses_overlap_solve. */
elses_status elses_spai_apply(elses_ctx ctx, elses_mat mat, const float *params, int32_t bf16, double *M_vals);
/* Learned preconditioner of the overlap solves (Sec. III-B: B^{-1} enters
 * every step of the generalized problem).  Runs the features, the network
 * (params: DEVICE FP32 [ELSES_MLP_PARAMS], BF16 inference if bf16 != 0) and
 * the assembly of M ~ B^{-1} on B's pattern (diagonal blocks symmetrised),
 * and keeps M with the matrix.  Region sets created afterwards carry M's
 * values with A and B (FP64, and FP32 for ELSES_MIXED), and their solves
 * with opts->precond use it; global solves with opts->precond use the device
 * copy of M kept here and the spectral interval of M B estimated here, once
 * (Lanczos in the B inner product; a non-positive lower end marks M as not
 * SPD).  params = NULL removes M.  Needs atom positions.
 * Errors: ELSES_ERR_INVALID_ARG for a non-finite network output. */
elses_status elses_mat_set_preconditioner(elses_ctx ctx, elses_mat mat, const float *params, int32_t bf16);
/* Work of the last solve on this context.  Compact region solves: sparse
 * products launched (A, B and M products, summed over the regions; per region
 * one product serves all of its columns) and the number of regions whose
 * preconditioned overlap solve fell back to the plain iteration.  Global
 * solves: products 0 (not counted), fallbacks 1 if opts->precond was asked
 * for and the matrix's M is not SPD, else 0.  (HOST outputs, each may be
 * NULL.) */
elses_status elses_ctx_solve_counts(elses_ctx ctx, int64_t *products, int64_t *fallbacks);
/* Overlap solve x = p(B) s for nvec right-hand sides (DEVICE double
 * [M][nvec], nvec a multiple of 64) to relative residual tol by Richardson
 * steps with Chebyshev roots.  With M_vals (from elses_spai_apply) the steps
 * are x_{k+1} = x_k + tau_k M (s - B x_k) on the spectral interval of M B
 * (estimated by Lanczos); if M is not SPD the plain iteration is used.
 * passes_out receives the number of sparse passes, bracket_out (HOST [2])
 * the interval used, used_precond 1 if M was used. */
elses_status elses_overlap_solve(elses_ctx ctx, elses_mat mat, const double *M_vals, double tol, int32_t nvec,
                                 const double *s, double *x, int32_t *passes_out, double *bracket_out,
                                 int32_t *used_precond);

/* FP32 products with the FP32 copies of a matrix created with ELSES_MIXED:
 * y = fl32(X) x with FP32 accumulation, X = A (which=0) or B (which=1);
 * x, y DEVICE float [M][nvec], nvec a positive multiple of 64; `variant` as
 * in elses_opts (the LDS-staged variants have no FP32 form).  These are the
 * products of the mixed-precision overlap solve (diagnostics and tests). */
elses_status elses_spmm32(elses_ctx ctx, elses_mat mat, int which, int32_t variant, int32_t nvec, const float *x,
                          float *y);

/*
 * Multiple Arnoldi method with analytic energy integration (paper Sec. III-B,
 * Eqs. 15-18).
 *
 * For each column j the generalized problem is restricted to the direct sum
 * of two Krylov spaces of A (Eq. 15):
 *     L_nu = K_{nu/2}(A; e_j) + K_{nu/2}(A; B^{-1} e_j),   nu even.
 * Rayleigh-Ritz of the pencil (A, B) on L_nu gives Ritz values eps_m and
 * B-orthonormal Ritz vectors v_m (m < dim_j <= nu; Eqs. 16-17), and the energy
 * integral of a projected quantity becomes a finite sum (Eq. 18):
 *     e_j^T rho X e_j = sum_m f(eps_m) (e_j^T v_m)(v_m^T X e_j).
 * B^{-1} e_j is the Richardson/Chebyshev overlap solve to inner_tol.  A Krylov
 * sequence that is exhausted (new direction below 1e-10 of its candidate)
 * stops early, so dim_j < nu for regions smaller than the subspace.
 *
 * Outputs (HOST, each may be NULL), per column in the order given:
 *   eps [n_cols][nu]  Ritz values, ascending in the first dim_j entries, 0 after;
 *   w_I, w_B, w_A [n_cols][nu]  (e_j^T v_m)(v_m^T X e_j) for X = I, B, A
 *                     (0 beyond dim_j): any f then gives Eq. 18 on the host;
 *   dim [n_cols]      subspace dimension dim_j;
 *   rho_out           rho_ij = sum_m f(eps_m)(e_i^T v_m)(v_m^T e_j) on the
 *                     column patterns (layout of elses_density_matrix) for the
 *                     Fermi function f(eps) = 1 / (1 + exp((eps - mu) / kT))
 *                     (kT = 0: step, 1/2 at mu);
 *   col_traces_out [n_cols][2]  e_j^T rho B e_j and e_j^T rho A e_j for that f.
 * Errors: ELSES_ERR_INVALID_ARG for nu odd or outside [2, 48], kT < 0,
 * non-finite mu, bad or duplicate columns; ELSES_ERR_OOM when the nu + 5
 * vector blocks of a batch do not fit.
 */
typedef struct {
    int32_t nu;        /* subspace dimension, even, 2..48 (the paper uses 30); the
                        * per-column work arrays then fit in 64 KB of LDS */
    int32_t variant;   /* pass variant as in elses_opts (0: default) */
    int32_t slots;     /* global solves: columns per batch, multiple of 64 (0: up to 1024) */
    double inner_tol;  /* overlap solve tolerance for B^{-1} e_j (<= 0: 1e-13) */
    double mu, kT;     /* Fermi function of rho_out and col_traces_out */
} elses_arnoldi_opts;
void elses_arnoldi_opts_default(elses_arnoldi_opts *o);
/* Global solve: columns cols[n_cols] (HOST, distinct) of the whole pencil. */
elses_status elses_arnoldi(elses_ctx ctx, elses_mat mat, int32_t n_cols, const int32_t *cols,
                           const elses_arnoldi_opts *o, double *eps, double *w_I, double *w_B, double *w_A,
                           int32_t *dim, double *rho_out, double *col_traces_out);
/* Region solve (real-space projection): every column of a region set on its
 * region's principal sub-pencil, outputs in the column order of
 * elses_regions_info (pattern rows outside the region hold 0). */
elses_status elses_regions_arnoldi(elses_ctx ctx, elses_regions reg, const elses_arnoldi_opts *o, double *eps,
                                   double *w_I, double *w_B, double *w_A, int32_t *dim, double *rho_out,
                                   double *col_traces_out);

/* Library version string. */
const char *elses_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ELSES_H */
