// Internal declarations of the gfx950 generalized shifted Krylov solver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/elses.h"

namespace elses {

constexpr int kWave = 64;         // CDNA wavefront width
constexpr int kBlock = 256;       // threads per workgroup for the direct passes
constexpr int kWavesPerBlock = kBlock / kWave;
// Staged passes: cluster shapes {atoms (= waves) per cluster, LDS rows of 64
// doubles}.  Shape 0 uses 147 KB of the 160 KB LDS (one workgroup per CU),
// shape 1 uses 72 KB (two workgroups per CU).
constexpr int kStageShapes = 2;
constexpr int kStageWaves[kStageShapes] = {8, 4};
constexpr int kStageRows[kStageShapes] = {288, 144};

// Atom-block sparse matrix on the device.  Atoms carry 4 or 1 orbitals, in
// any order.  Internally the blocks of row atom I are reordered so that the
// 4-orbital neighbours come first: a 4-wide part [brow[I], bsplit[I]) and a
// 1-wide part [bsplit[I], brow[I+1]), each in ascending neighbour order.  The
// values of row I are contiguous from voff[I] in that order, each block
// n_I x n_J row-major.  The asc_* arrays describe the same blocks in the
// caller's (ascending) order, for output patterns.
struct DevMatrix {
    int n_atoms = 0, M = 0;
    int nnzb = 0;
    int64_t nnz = 0;
    int *atom_off = nullptr;  // [n_atoms+1] first orbital of each atom
    int *orb_atom = nullptr;  // [M] atom of each orbital
    int *brow = nullptr;      // [n_atoms+1]
    int *bsplit = nullptr;    // [n_atoms]
    int *borb = nullptr;      // [nnzb] first orbital of the coupled atom (internal order)
    int64_t *voff = nullptr;  // [n_atoms]
    int *asc_borb = nullptr;  // [nnzb] ascending order: first orbital of the coupled atom
    int *asc_n = nullptr;     // [nnzb] ascending order: its orbital count
    int64_t *asc_voff = nullptr;  // [nnzb] ascending order: value offset of the block
    double *A = nullptr, *B = nullptr;  // [nnz] internal layout
    float *A32 = nullptr, *B32 = nullptr;
    // clusters of consecutive atoms for the LDS-staged passes, per shape
    struct Clusters {
        int n = 0;            // 0: shape unavailable
        int *atom = nullptr;  // [n+1] first atom of each cluster
        int *uoff = nullptr;  // [n+1] offsets into urow
        int *urow = nullptr;  // union of coupled orbitals of each cluster (ascending)
        int *bloc = nullptr;  // [nnzb] internal order: LDS row of the coupled atom's first orbital
    } cl[kStageShapes];
    // Row groups for the grouped passes: a 4-orbital atom with up to
    // kGroupH 1-orbital atoms it couples to most strongly (or a single atom).
    // A group's rows share one gather of the union of their coupled atoms;
    // its values are dense R x n_J blocks over that union (zero where a
    // member does not couple), 4-orbital union atoms first.
    struct Groups {
        int n = 0;
        int *R = nullptr;         // [n] rows of each group (1, 4..4+kGroupH)
        int *roff = nullptr;      // [n+1] offsets into rows
        int *rows = nullptr;      // member orbitals: the 4-orbital atom's rows, then each H row
        int *uoff = nullptr;      // [n+1] offsets into uorb
        int *u4 = nullptr;        // [n] end of the 4-orbital part of the union
        int *uorb = nullptr;      // first orbital of each union atom
        int64_t *voff = nullptr;  // [n] value offset of the group's dense blocks
        double *A = nullptr, *B = nullptr;
        float *A32 = nullptr, *B32 = nullptr;  // FP32 copies (mixed precision)
        int64_t nval = 0;
    } grp;
};

constexpr int kGroupH = 4;

struct HostMatrix {
    int n_atoms = 0, M = 0;
    std::vector<int> atom_off, brow, bcol;  // caller's ascending block order
    std::vector<double> pos;
    double box = 0;
    int pmax = 0;                     // max over atoms of the coupled-orbital count
    std::vector<int> atom_plen;       // coupled-orbital count per atom
    // caller's layout (caller matrices only; used to carve regions)
    std::vector<int8_t> n_orb;
    std::vector<int64_t> in_voff;     // value offset of each block (ascending order), nnzb + 1
    std::vector<double> A_in, B_in;
    std::vector<double> M_in;         // learned preconditioner on B's pattern (caller layout), or empty
    std::vector<int> grp_row0;        // first row of each row group
};

}  // namespace elses

struct elses_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int n_cu = 256;
    // sampled timing of the Chebyshev pass
    int prof_stride = 0;
    int64_t prof_launches = 0;
    double prof_ms = 0.0;
    double prof_bytes = 0.0;
    double prof_flops = 0.0;
    double prof_bytes_acc = 0.0;  // compact region launches: sums over the timed launches
    double prof_flops_acc = 0.0;
    // profiled compact solves: summed share of resident workgroup time without a region
    double prof_idle_acc = 0.0;
    int64_t prof_idle_n = 0;
    int64_t total_passes = 0;
    int prof_slots = 0;
    // last compact region solve: sparse products launched (A, B, M; summed over
    // regions) and regions whose preconditioned overlap solve fell back
    int64_t last_products = 0;
    int64_t last_fallbacks = 0;
};

struct elses_mat_s {
    elses_ctx ctx = nullptr;
    int precision = ELSES_FP64;
    elses::HostMatrix h;
    elses::DevMatrix d;
    double b_lo = 0, b_hi = 0;  // interval enclosing the spectrum of B
    // learned preconditioner (elses_mat_set_preconditioner): M in the internal
    // value layout (device, FP64), the interval of M B, and whether M is SPD
    double* M_dev = nullptr;
    double mb_lo = 0, mb_hi = 0;
    bool mb_spd = false;
    // autotuned pass variant and slot count per precision (0 FP64, 1 mixed);
    // slots 0: not tuned
    int tuned_variant[2] = {0, 0};
    int tuned_slots[2] = {0, 0};
};

namespace elses {

// ---------------------------------------------------------------------------
// Vector passes over the atom-block matrix (lanes = right-hand sides).
// ---------------------------------------------------------------------------
enum PassKind {
    PASS_LANCZOS_A = 0,     // w = A q_n, s' = w - beta_{n-1} t_{n-1}, partial q_n.s'
    PASS_STEP = 1,          // Richardson step x_{k+1} = x_k + tau (s - B x_k)
    PASS_STEP_LAST = 2,     // last step, partial v.s and s.s
    PASS_PLAIN = 3,         // y = X x
    // mixed precision: FP32 matrix values; overlap solve in FP32 vectors with
    // one FP64-accumulated residual refinement
    PASS_LANCZOS_A_MX = 4,  // as PASS_LANCZOS_A with FP32 values
    PASS_STEP32 = 5,        // FP32 Richardson step
    PASS_REFINE = 6,        // r = s - B x (FP64 accumulation); FP32 r and first correction iterate
    PASS_STEP32_LAST = 7,   // last FP32 correction step, v = x + d, partial v.s and s.s
    PASS_PLAIN32 = 8,       // y = X x in FP32 (diagnostics)
    PASS_STEP_FIRST = 9,    // s = s' - alpha_n t_n, x_1 = g0 s formed while gathering; first step
    PASS_STEP32_FIRST = 10, // the same with an FP32 iterate; also writes s in FP32
    // preconditioned overlap solve x_{k+1} = x_k + tau M (s - B x_k)
    PASS_RESID = 11,        // r = s - B x  (S: s, gathered: x, out: r)
    PASS_PSTEP = 12         // x_{k+1} = x_k + tau M r  (S: x_k, gathered: r, values: M)
};
constexpr int kPassKinds = 13;

struct PassArgs {
    // matrix
    const int *atom_off;
    const int *brow;
    const int *bsplit;
    const int *borb;
    const int64_t *voff;
    const double *vals;
    const float *vals32;   // FP32 values of the same matrix (mixed kinds)
    int n_atoms;
    // layout: vectors are [M][ld] doubles, ld = slot count.  Direct passes:
    // slabs are groups of atoms_per_slab consecutive atoms (one per wave).
    // Staged passes: the groups are the clusters.  n_slabs (groups) is a
    // multiple of 8; trailing groups may be empty.
    int ld;
    int n_slabs, atoms_per_slab, n_tiles;
    int n_tiles32;  // column tiles of the passes over FP32 vectors
    int staged;  // 0: direct gathers; 1 + s: LDS-staged with cluster shape s; 9: row groups
    int n_clusters;
    const int *cl_atom, *cl_uoff, *cl_urow, *bloc;
    int n_grp, group_split;  // row groups; waves sharing one group (1, 2 or 4)
    // Region tiles (block-diagonal batched matrix, grouped passes only):
    // slab_group[slab * groups_per_slab + i] is the i-th group of a slab or -1,
    // slab_tile[slab] the column tile whose per-slot state the slab uses.  The
    // vectors are [M][ld] with ld = the tile width; every row belongs to one
    // tile.  mask[row * mask_words + w] holds one bit per column: set when the
    // row lies inside that column's region.  Outputs outside it are zero.
    const int *slab_group, *slab_tile;
    const uint64_t *mask;
    int mask_words;
    const int *tile_live;  // region tiles: columns of each tile still running (0: the tile is skipped)
    int place;               // workgroup placement (0 XCD regions tile by tile, 1 XCD regions tile-fastest, 2 plain)
    const int *g_R, *g_roff, *g_rows, *g_uoff, *g_u4, *g_uorb;
    const int64_t *g_voff;
    // vectors
    const double *Xg;   // gathered operand
    double *Xio;        // STEP*: out x_{k+1} (STEP_LAST, STEP32_LAST: v); PLAIN: out y
    double *S;          // LANCZOS_A: in t_{n-1} / out s'; STEP*_FIRST: in s' (gathered);
                        // STEP, STEP_LAST, REFINE, STEP32_LAST: in s
    double *Sout;       // STEP*_FIRST: out s = s' - alpha_n t_n
    const double *Vq;   // LANCZOS_A: q_n (unnormalised)
    const double *Tn;   // STEP*_FIRST: t_n (unnormalised, gathered)
    // FP32 vectors of the mixed-precision overlap solve
    const float *Xg32;  // gathered FP32 operand (STEP32*, REFINE, PLAIN32)
    float *Xio32;       // FP32 output iterate
    const float *R32;   // FP32 right-hand side (STEP32*)
    float *R32o;        // STEP32_FIRST: FP32 s; REFINE: FP32 residual
    const float *Xr1;   // STEP32_LAST: first-round FP32 solution x
    // per-slot scalars
    const double *inv_beta;   // 1/beta_{n-1}
    const double *coefT;      // beta_{n-1}/beta_{n-2}
    const double *alpha;      // alpha_n (reduced before the first step)
    const int *slot_n;        // iteration counter (0 = start vector)
    const int *slot_row;      // e_j row of the slot's column (-1 idle)
    // Richardson step x_{k+1} = x_k + tau (s - B x_k)
    double tau;
    double g0;                // x_1 = g0 * s
    // dot partials [n_slabs][ld]
    double *part0, *part1;
};

void launch_pass(PassKind kind, const PassArgs &a, hipStream_t st);
// s = s' - alpha_n t_n and x_1 = g0 s, element-wise over [M][vw] (FP32 copies when S32 != null)
void launch_overlap_start(int M, int vw, const double *Sp, const double *Tn, const double *alpha,
                          const double *inv_beta, const int *row_tile, double g0, double *S, double *X1, float *S32,
                          float *X132, hipStream_t st);

// ---------------------------------------------------------------------------
// Per-slot shift recurrences and bookkeeping.
// ---------------------------------------------------------------------------
struct ShiftArgs {
    int ld;          // slot count
    int vld;         // row stride of the [M][vld] vectors; slot s uses column s % vld
    int K;           // shifts
    int M;
    const double *z; // [K] complex
    const double *cw; // [K] complex weights for rho (density mode) or null
    // per-slot state
    int *slot_n;
    int *slot_row;    // e_j row (-1 idle)
    int *slot_cidx;   // index into the column list
    double *beta_prev;
    double *inv_beta;
    double *coefT;
    const double *alpha;
    const double *vs, *ss;         // v.s and s.s per slot (reduced)
    double *eta, *zeta;            // [ld][K] complex
    int *conv;                     // [ld][K] iteration of convergence, 0 active
    double *res;                   // [ld][K]
    double *xs, *ps;               // [ld][K][rmax] complex
    int rmax;                      // row capacity per slot
    const double *Vq;              // q_n buffer (unnormalised)
    // column bookkeeping
    int n_cols;
    const int *cols;               // [n_cols] global column (orbital) index
    const int64_t *row_off;        // [n_cols+1] offsets into rows (pattern mode)
    const int *rows;               // pattern rows (pattern mode) or null (full: 0..M-1)
    const int64_t *vidx;           // value index of B_ji / A_ji per pattern entry (density)
    const double *Bv, *Av;         // FP64 values (density traces)
    int full;                      // 1: rows are 0..M-1
    double tol;
    int max_outer;
    const int *slot_map;           // initial column of each slot (-1 idle), or null: slot s takes column s
    int *tile_live;                // region tiles: running columns per tile of vld slots (or null)
    int *queue;                    // next column to start
    int *remaining;                // columns not yet finished
    int *n_notconv;                // columns finished without convergence
    // outputs
    double *x_out;                 // may be null
    int *iters_out;                // may be null
    double *resid_out;             // may be null
    double *rho_out;               // density mode (may be null)
    double *ctr_out;               // [n_cols][2] per-column traces (may be null)
};

// out[c] = sum over n_part partial rows (deterministic, two stages; tmp holds
// ceil(n_part/64) x ld doubles).  With slot_n given, idle or starting slots get 0.
void launch_col_reduce(const double *part, int n_part, int ld, double *tmp, const int *slot_n, const int *slot_row,
                       double *out, hipStream_t st);
// Region tiles: out[t * L + c] = sum over the slabs of tile t of part[slab * L + c],
// in two deterministic stages.  Chunk k covers slabs [chunk_s0[k], chunk_s1[k]);
// tile t owns chunks [tile_chunk_off[t], tile_chunk_off[t+1]); tmp holds
// n_chunks x L doubles.
void launch_col_reduce_tiles(const double *part, int L, int n_tiles, int n_chunks, const int *chunk_s0,
                             const int *chunk_s1, const int *tile_chunk_off, double *tmp, const int *slot_n,
                             const int *slot_row, double *out, hipStream_t st);
void launch_shift_update(const ShiftArgs &a, hipStream_t st);
void launch_pattern_setup(const DevMatrix &m, int n_cols, const int *cols, const int64_t *row_off, int *rows,
                          int64_t *vidx, hipStream_t st);
void launch_slot_init(const ShiftArgs &a, int n_active, hipStream_t st);

// Generic products used by setup, audits and diagnostics: y = X x (nvec vectors, [M][ld]).
void launch_spmm_generic(const DevMatrix &m, const double *vals, int nvec, int ld, const double *x, double *y,
                         hipStream_t st);
// Complex true residual ||e_j - (z_k B - A) x_{c,k}||_2 for full-mode outputs,
// with the FP64 values or (fp32_values) the FP32 values of a mixed matrix.
void launch_true_residual(const DevMatrix &m, bool fp32_values, int n_cols, const int *cols, int K,
                          const double *z, const double *x_full, double *res_out, hipStream_t st);
void launch_sum_pairs(const double *v, int n, double *out2, hipStream_t st);
// rho, per-column traces and per-(column, coupled atom) ICOHP from stored pattern-mode x
void launch_reweight(int n_cols, int K, const double *cw, const int64_t *pat_off, const int64_t *vidx,
                     const int64_t *blk_off, const int64_t *pbo, const double *Bv, const double *Av,
                     const double *x, double *rho, double *ctr, double *icohp, hipStream_t st);

// Partial dot products (deterministic two-stage): out[b] = sum over block b
void launch_dot_partial(const double *a, const double *b, int n, double *part, int nblocks, hipStream_t st);
// out = a x + b y over n values (x may be null when a == 0)
void launch_axpby(int64_t n, double a, const double *x, double b, const double *y, double *out, hipStream_t st);
// per column c of [M][ld] blocks v, s: part0[g][c] = sum of v s and part1[g][c] = sum of s s
// over the rows of chunk g (n_groups equal chunks, fixed order)
void launch_dots2_partial(int M, int ld, int n_groups, const double *v, const double *s, double *part0,
                          double *part1, hipStream_t st);

// Learned SPAI (spai.hip): features, exact-inverse targets, FP32 training,
// BF16 inference, assembly of M on B's pattern.
void launch_spai_features(int64_t n, const int *pI, const int *pJ, const int *pb, const DevMatrix &d,
                          const int *bcol, const double *pos, double box, float *feat, hipStream_t st);
void launch_eye(int M, int ld, int c0, double *S, hipStream_t st);
void launch_spai_targets(int64_t n, const int *pI, const int *pJ, const int *atom_off, const double *X, int ld,
                         int c0, float *target, float *mask, hipStream_t st);
void launch_gemm(int Mr, int N, int K, const float *A, int64_t sa0, int64_t sa1, const float *B, int64_t sb0,
                 int64_t sb1, float *C, int64_t sc0, bool acc, hipStream_t st);
void launch_bias_act(int64_t rows, int N, float *Z, const float *b, float *H, bool act, hipStream_t st);
void launch_gelu_back(int64_t n, const float *Z, float *G, hipStream_t st);
void launch_colsum(int64_t rows, int N, const float *G, float *db, hipStream_t st);
void launch_loss(int64_t n, const float *out, const float *T, const float *W, float *gout, double *part,
                 double *loss, float *scale, hipStream_t st);
void launch_adam(int64_t n, float *th, const float *g, float *m, float *v, float lr, int t, hipStream_t st);
void launch_gather_rows(int n, int F, const int *idx, const float *src, float *dst, hipStream_t st);
void launch_to_bf16(int64_t n, const float *x, uint16_t *y, hipStream_t st);
void launch_infer_bf16(int64_t n, const uint16_t *Wbf, const float *params, const float *feat, float *out,
                       hipStream_t st);
void launch_spai_assemble(int64_t n, const int *pI, const int *pJ, const int *pb, const int *pbt,
                          const DevMatrix &d, const float *out, double *Mv, hipStream_t st);

// Region problems in the compact per-region layout (region.hip): one
// workgroup of kRegThreads threads solves one region at a time; the regions
// come from a device queue.  See region.hip for the layout.
constexpr int kRegThreads = 512;

struct RegionDesc {
    int m;         // orbitals of the region
    int nslice;    // slices of 64 positions (P = 64 nslice)
    int slice0;    // first slice in the slice tables
    int col0;      // first column of the region in the column list
    int ncol;      // columns solved (1..4)
    int cw;        // column width of the region's vectors: 1, 2 or 4 (>= ncol)
    int64_t ent0;  // first entry of the region's slices
    int64_t pos0;  // first position in the position tables
    int64_t hent0; // first entry of the region's slices in the half layout of B (mixed precision)
    int heb;       // |B_pq| < 2^(heb - L) over the half layout's entries, where no position takes
                   // more than 2^L - 1 transpose terms (fixed-point scale of its products)
};

struct CompactArgs {
    const RegionDesc* reg;
    const int* order;        // queue order of the regions (costliest first: nonzeros x sqrt(kappa of B))
    int n_regions;
    const int* slice_len;    // longest row of each slice
    const int* slice_ent;    // first entry of each slice, relative to its region
    const uint16_t* idx;     // entries: column position inside the region
    const double *A64, *B64; // entries: FP64 values
    const float *A32, *B32;  // entries: FP32 values (mixed precision)
    const double* M64;       // entries: learned preconditioner M (precond launches), FP64
    const float* M32;        //          and its FP32 copy (mixed precision)
    const uint16_t* pos_row; // region orbital of each position (>= m: padding)
    // half layout of B (FP32): each off-diagonal pair {p, q} stored once, in
    // the row of p when p + q is even and p < q or odd and p > q; diagonal apart
    int half;                // 1: the FP32 Richardson steps use the half layout
    const int* hslice_len;   // longest half row of each slice
    const int* hslice_ent;   // first half entry of each slice, relative to its region
    const uint16_t* hidx;    // half entries: column position inside the region
    const float* hval;       // half entries: FP32 values of B
    const float* hdiag;      // [positions] FP32 diagonal of B (0 on padding)
    const int* col_pos;      // [n_cols] position of the column's unit vector
    const int64_t* pat_off;  // [n_cols+1] pattern offsets (caller's layout)
    const int* pat_pos;      // position of each pattern entry (-1 outside the region)
    const double *pat_B, *pat_A;  // B_ji, A_ji of each pattern entry (traces)
    const int64_t* carry_off;     // [n_cols] first carried entry of each column (x, p: [K][len])
    const int* carry_full;        // [n_cols] 1: carried on every position of its region
    const int64_t* full_off;      // [n_cols] first orbital of each column's full output block
    int full_out;                 // x_out holds [K][m] region vectors per column
    int audit;                    // resid_out of fully carried columns = FP64 true residual
    int K;
    const double* z;
    const double* cw;
    double tol;
    int max_outer;
    // Richardson plan of each region (per round, on its own overlap interval):
    // degree, first step, and the inverse roots of steps 1 .. d-1 at rtau[r * tau_stride]
    const int* rdeg;
    const double* rg0;
    const double* rtau;
    int tau_stride;
    int lds_half;                 // > 0: a second LDS iterate buffer starts this many values after the
                                  // first (Richardson steps ping-pong in LDS); 0: staged through vec
    double inner_tol;             // overlap solve tolerance (preconditioned CG: per round)
    int inner_max;                // preconditioned CG steps per round before the fallback
    unsigned long long* products; // sparse products launched (A, B and M), summed over regions
    int* n_fallback;              // regions whose preconditioned overlap solve fell back
    double* vec;                  // per workgroup: six [Pmax][Cmax] FP64 blocks
    size_t vec_stride;
    double *eta, *zeta, *res, *fac;  // [n_cols][K] (x2, x2, x1, x4)
    int* conv;                       // [n_cols][K] iteration of convergence, 0 running
    double *xs, *ps;                 // carried x and p (complex)
    int* queue;
    unsigned long long* wg_clock;    // profiled launches: [n_wg][2] start and end stamps (wall clock), else null
    int* n_notconv;
    double* x_out;
    int* iters_out;
    double* resid_out;
    double* rho_out;
    double* ctr_out;
};
// resident workgroups per CU of the kernel for (precision, column width, preconditioned, LDS bytes)
int compact_occupancy(bool fp64, int cw, bool precond, size_t lds);
// one persistent launch over the regions a.order[0 .. a.n_regions) (all of column width cw)
void launch_compact(const CompactArgs& a, bool fp64, int cw, bool precond, int n_wg, size_t lds, hipStream_t st);

// n ints set to zero by a kernel (no memset node, so the call can be captured)
void launch_zero_ints(int* p, size_t n, hipStream_t st);

// idx-th smallest eigenvalue of the symmetric tridiagonal matrix with
// diagonal a and off-diagonal b (Sturm-sequence bisection).
double tri_eig(const std::vector<double>& a, const std::vector<double>& b, int idx);

// Chebyshev-Richardson plan for B v = s on an interval [lo, hi] holding B's
// spectrum: degree d (the smallest with 1/T_d(c/h) <= tol, c and h the
// interval's centre and half width, at least 3, at most kRichMaxDegree), the
// first step g0 = 1/theta_0 and the inverse roots tau_k = 1/theta_k of the
// later steps, the roots theta of T_d on the interval in Leja order.
struct Rich {
    int d = 2;
    double g0 = 0;
    std::vector<double> tau;  // steps k = 1 .. d-1
    double reached = 0;       // 1/T_d(c/h): the residual factor the plan guarantees on [lo, hi]
};
constexpr int kRichMaxDegree = 400;
Rich richardson_plan(double lo, double hi, double tol);

// Host-side construction of the compact layout (region_host.hip).
struct CompactHost {
    std::vector<RegionDesc> reg;
    std::vector<int> slice_len, slice_ent;
    std::vector<uint16_t> idx, pos_row;
    std::vector<double> A64, B64, M64;
    std::vector<float> A32, B32, M32;
    std::vector<int> hslice_len, hslice_ent;  // half layout of B (mixed precision)
    std::vector<uint16_t> hidx;
    std::vector<float> hval, hdiag;
    std::vector<int64_t> region_hnnz;         // stored off-diagonal pairs of each region's half layout
    std::vector<int> cols;      // global orbital of each column, region by region
    std::vector<int> col_pos;   // position of each column's unit vector in its region
    std::vector<int> col_region;
    std::vector<int64_t> pat_off;
    std::vector<int> pat_pos;
    std::vector<double> pat_B, pat_A;
    std::vector<int> region_orbs;
    std::vector<int64_t> region_nnz;   // nonzeros of each region's matrices
    std::vector<double> ritz_lo, ritz_hi;  // extreme Ritz values of each region's B (Lanczos)
    int max_slices = 0;
    int64_t useful = 0;
    size_t lds_fp64 = 0, lds_fp32 = 0;  // LDS of the largest region (P x cw values)
};
// Carve the regions (atoms within radii[r] of centres[r], minimum image) and
// build their compact layout.  orb_mask (may be null) selects the centre's
// orbitals solved as columns (bit q: orbital q; 0 or null: all).  The
// learned preconditioner's values (h.M_in, when set) are carved alongside A
// and B.  Returns an error message or null.
const char* build_compact(const HostMatrix& h, int n_regions, const int* centres, const double* radii,
                          const uint8_t* orb_mask, bool want32, CompactHost& out);

// Multiple Arnoldi method (arnoldi.hip).  Vector blocks are [rows][Lw]; row
// chunks (ch_r0, ch_r1, ch_seg) lie inside one segment each, seg_ch0 lists
// each segment's chunks; partials are [chunk][K][Lw], per-slot results
// [slot][K] with slot = segment * Lw + lane.
enum MaBookOp { MA_BOOK_START = 0, MA_BOOK_FIRST, MA_BOOK_SECOND, MA_BOOK_NORM0, MA_BOOK_GAMMA, MA_BOOK_NORM1,
                MA_BOOK_LAST };
void launch_ma_dots(int nc, const double *cand, size_t cstride, const double *W, size_t wstride, int nq, int Lw,
                    int n_chunks, const int *ch_r0, const int *ch_r1, double *part, int K, hipStream_t st);
void launch_ma_reduce(const double *part, int K, int Lw, int n_seg, const int *seg_ch0, double *out, hipStream_t st);
void launch_ma_update(int nc, double *cand, size_t cstride, const double *W, size_t wstride, int nq, int Lw,
                      int n_chunks, const int *ch_r0, const int *ch_r1, const int *ch_seg, const double *coef, int K,
                      int stats, double *part, hipStream_t st);
void launch_ma_vec(int op, double *D, const double *X, const double *Y, int Lw, int n_chunks, const int *ch_r0,
                   const int *ch_r1, const int *ch_seg, const double *s, int s_stride, double *part, hipStream_t st);
void launch_ma_unit(int n_slots, int Lw, const int *slot_row, double *W0, hipStream_t st);
void launch_ma_book(int op, int b, int nu, int nq, int K, const double *coef, double *H, double *Br, double *stt,
                    unsigned long long *dead, const int *slot_row, int n_slots, hipStream_t st);
void launch_ma_eig(int n_slots, int nu, const double *H, const double *Br, const unsigned long long *dead,
                   const int *slot_row, const int *slot_col, const double *W, size_t wstride, int Lw, double mu,
                   double kT, double *eps, double *wI, double *wB, double *wA, int *dim, double *g, double *ctr,
                   hipStream_t st);
void launch_ma_rho(int n_cols, const int64_t *pat_off, const int *rows, const int *col_slot, const double *g, int nu,
                   const double *W, size_t wstride, int Lw, double *rho, hipStream_t st);

}  // namespace elses
