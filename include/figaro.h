/*
 * figaro.h -- C ABI of the MI355X (gfx950) two-table Figaro library.
 *
 * The library computes, for two tables A (m1 x n1) and B (m2 x n2) and
 * their int32 join keys, the upper-triangular factor R of the QR
 * decomposition of the join matrix J and the singular values of J, without
 * materialising J ("Figaro on GPUs: Two Tables", Section 1: Theory, the QR
 * head/tail operators and Claim 1; Experiments section for the R/sigma
 * pipeline).  J is the natural join of A and B on their keys: the rows
 * [A_r | B_s] for every pair with key_A[r] == key_B[s]; with no keys it is
 * the Cartesian product A x B (Section 1).
 *
 * Conventions shared by every entry point:
 *   - Pointers named "device" point to GPU memory; everything else is host.
 *   - All memory is allocated and owned by the caller.  The library never
 *     frees caller memory and allocates nothing on the compute path of
 *     figaro_r and figaro_sigma; a plan allocates its launch tables (and its
 *     graph) once per buffer triple, on that triple's first execution.
 *   - Calls enqueue work on `stream` (a hipStream_t passed as void*; NULL is
 *     the default stream) and return without waiting, except those marked
 *     "synchronous".
 *   - Matrices are row-major with a leading dimension `ld` (elements, >= cols).
 *   - Return values are FIGARO_* codes; no exception crosses the ABI.  The
 *     message of the last failure on the calling thread is available from
 *     figaro_last_error().
 *   - Calls that share one workspace race when they overlap on a device.
 */
#ifndef FIGARO_H
#define FIGARO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------- codes */
#define FIGARO_OK 0
#define FIGARO_EINVAL (-1)      /* invalid argument (null pointer, ld < cols, dtype mismatch, N = 0, keys on one side only, unsupported width or route) */
#define FIGARO_EUNSORTED (-2)   /* keys not non-decreasing (detected on the device, reported by figaro_status) */
#define FIGARO_EWORKSPACE (-3)  /* workspace smaller than the size query returned */
#define FIGARO_EHIP (-4)        /* HIP runtime error; see figaro_last_error() */
#define FIGARO_ETIMEOUT (-5)    /* a bounded device-side wait expired (reported by figaro_status) */

/* element types */
#define FIGARO_F32 0
#define FIGARO_F64 1

/* precision of the QR reduction */
#define FIGARO_PLAIN_FP64 0        /* every stage in FP64 (FP32 inputs are widened exactly) */
#define FIGARO_MIXED_FP32 1        /* compact matrix stored and reduced in FP32 (FP64 scans, FP64 reflector scalars, FP64 root) */
#define FIGARO_MIXED_FP32_REFINE 2 /* FIGARO_MIXED_FP32 followed by one FP64 refinement sweep against the exact Gram matrix */

/*
 * Flag OR'ed into `precision`: the two-sided form.  Each group's region-1
 * rows [sqrt(m2_g) A_r | H(B_g)] are themselves replaced by their QR head
 * and tail (the faster variant noted after Claim 1: the head operator is
 * applied to both tables), giving per group one head row
 * [sqrt(m2_g) H(A_g) | sqrt(m1_g) H(B_g)], m1_g - 1 rows [sqrt(m2_g) T(A_g) | 0]
 * and the m2_g - 1 rows [0 | sqrt(m1_g) T(B_g)].  Same R, fewer flops.
 */
#define FIGARO_TWO_SIDED 0x100

/*
 * Flag OR'ed into `precision` (FP64 only): the Givens route.  After Claim 1,
 * the compact matrix is reduced by Givens rotations entry by entry (Section 1:
 * the continuation of Claim 1), in place of Householder reflectors: every
 * region's rows are absorbed one at a time into the triangle of their leaf by
 * plane rotations (one wave per leaf), and the leaves' triangles are merged the
 * same way in a binary tree.  The root merges are those of the other routes.
 * Every region must be at most 64 columns wide (the tails, and region 1 / the
 * head rows of a natural join), else FIGARO_EINVAL.
 */
#define FIGARO_GIVENS 0x200

/* largest supported join width N = n1 + n2 */
#define FIGARO_MAX_N 512

/*
 * One input table.
 *   data  device, rows x cols, row-major, leading dimension ld, element type dtype.
 *   keys  device, `rows` int32 join keys, non-decreasing (the paper's inputs
 *         are sorted by the join attribute, Experiments section); NULL on both
 *         tables selects the Cartesian product.
 */
typedef struct figaro_table {
    const void *data;
    int64_t rows, cols, ld;
    int32_t dtype;
    const int32_t *keys;
} figaro_table;

/*
 * Workspace bytes needed by figaro_r / figaro_compact for these shapes
 * (host-only, no device access).  The size is an upper bound that does not
 * depend on key values.  Returns FIGARO_EINVAL for invalid shapes.
 */
int figaro_r_workspace_size(const figaro_table *A, const figaro_table *B, int32_t precision,
                            size_t *bytes);

/*
 * R of the join matrix (Section 1, Claim 1 and the QR step of the Experiments
 * section).  Stages, all on the device: key grouping; per-group QR head and
 * tail of B as scaled prefix sums (head H, tail T of Section 1); assembly of
 * the compact matrix
 *     region 1, one row per matched A row r of group g:  [ sqrt(m2_g) A_r | H(B_g) ]
 *     region 2, m2_g - 1 rows per group:                [ 0 | sqrt(m1_g) T(B_g) ]
 * Householder TSQR of the compact matrix; rows of R normalised to a
 * non-negative diagonal (a negative diagonal negates the row, a zero
 * diagonal negates it iff its first nonzero is negative, -0.0 becomes +0.0).
 *   R     device, FP64, N x N row-major with leading dimension ldr >= N;
 *         fully written (zeros below the diagonal).
 *   ws    device workspace of at least figaro_r_workspace_size() bytes,
 *         256-byte aligned.  After the call it holds the group table and
 *         the device status word (read with figaro_status).
 * An empty join (no common key) gives R = 0.  Unsorted keys give
 * FIGARO_EUNSORTED from figaro_status; no group is then formed (G = 0) and
 * R = 0.
 */
int figaro_r(const figaro_table *A, const figaro_table *B, int32_t precision,
             double *R, int64_t ldr, void *ws, size_t ws_bytes, void *stream);

/*
 * Only the first stages of figaro_r: grouping, head/tail scan and assembly.
 * Leaves the group table and the compact matrix in `ws` (locate them with
 * figaro_inspect).  For tests and diagnostics.
 */
int figaro_compact(const figaro_table *A, const figaro_table *B, int32_t precision,
                   void *ws, size_t ws_bytes, void *stream);

/*
 * Device addresses, inside `ws`, of the intermediate results of
 * figaro_compact / figaro_r for these shapes (host-only, no device access).
 *   counts    int64[4]: G (groups), R1 (region-1 rows), R2 (region-2 rows),
 *             join_rows (sum over groups of m1_g * m2_g)
 *   group     int32 arrays of capacity group_cap: key, offA, m1, offB, m2, r1, r2
 *             (r1_g, r2_g are the first rows of group g in regions 1 and 2)
 *   heads     FP64, group_cap x n2: H(B_g)
 *   m1        Claim 1 form: region 1, R1 rows x N, ld = N;
 *             two-sided form: the G head rows, G x N, ld = N
 *   m2        region 2, R2 rows x n2 (the zero block is implicit), ld = n2
 *   heads_a   two-sided form only (else NULL): FP64, group_cap x n1, H(A_g)
 *   tails_a   two-sided form only (else NULL): (R1 - G) x n1, ld = n1,
 *             rows sqrt(m2_g) T(A_g) of group g from row r1_g - g
 *   m_dtype   element type of m1, m2 and tails_a (FIGARO_F64 for
 *             FIGARO_PLAIN_FP64, FIGARO_F32 otherwise)
 *   status    int32[1], device status word
 */
typedef struct figaro_view {
    int64_t *counts;
    int32_t *g_key, *g_offA, *g_m1, *g_offB, *g_m2, *g_r1, *g_r2;
    int64_t group_cap;
    double *heads;
    void *m1, *m2;
    double *heads_a;
    void *tails_a;
    int32_t m_dtype;
    int32_t *status;
} figaro_view;

int figaro_inspect(const figaro_table *A, const figaro_table *B, int32_t precision,
                   void *ws, size_t ws_bytes, figaro_view *out);

/*
 * Workspace bytes needed by figaro_sigma, figaro_sigma_jacobi and
 * figaro_sigma_bidiag for an n x n R.
 */
int figaro_sigma_workspace_size(int64_t n, size_t *bytes);

/*
 * Singular values of R (equal to those of the join matrix; Related Works: SVD
 * through QR), descending, in FP64: by the bidiagonal route of
 * figaro_sigma_bidiag for n <= 128 and by the block one-sided Jacobi of
 * figaro_sigma_jacobi for 128 < n <= 512.  Arguments, workspace and errors as
 * those two.
 */
int figaro_sigma(const double *R, int64_t n, int64_t ldr, double *sigma,
                 void *ws, size_t ws_bytes, void *stream);

/*
 * The singular values by one-sided (Hestenes) Jacobi in FP64: rotations on
 * column pairs in a parallel (round-robin) order until a sweep finds every pair
 * orthogonal to |c_p . c_q| <= n 2^-53 |c_p||c_q| (at most 60 sweeps).
 * n <= 128: one workgroup with R in LDS; 128 < n <= 512: block Jacobi over
 * blocks of 16 columns, one workgroup per block pair, with bounded grid-wide
 * waits between rounds.  R is scaled by a power of two first (exact), so
 * squared norms stay in range.
 *   R      device, FP64, n x n, leading dimension ldr (any square matrix is accepted).
 *   sigma  device, FP64, n values, descending (NaN if a bounded wait expired).
 *   ws     device workspace of figaro_sigma_workspace_size() bytes, 256-byte
 *          aligned; afterwards its first int32 holds the number of sweeps
 *          (-1 if a bounded wait expired).
 * FIGARO_EINVAL for n outside [1, 512], NULL pointers, ldr < n or a misaligned
 * workspace; FIGARO_EWORKSPACE if ws_bytes is too small.
 */
int figaro_sigma_jacobi(const double *R, int64_t n, int64_t ldr, double *sigma,
                        void *ws, size_t ws_bytes, void *stream);

/*
 * The singular values by the route of a dense SVD (the paper's SVD of R):
 * Householder bidiagonalisation B = U^T R V by one wavefront (R in LDS;
 * reflector k on column k, then on row k, with the TSQR's reflector
 * conventions), then the singular values of the bidiagonal as the positive
 * eigenvalues of its Golub-Kahan tridiagonal (zero diagonal, off-diagonals
 * d1, e1, d2, ...) by multisection on Sturm counts, one workgroup per value
 * and 256 points per round, to an interval below 2^-53 of the Gershgorin
 * bound.  n <= 128 (FIGARO_EINVAL above).  Arguments, workspace and errors as
 * figaro_sigma_jacobi (the sweep count is set to 0); the workspace also
 * carries the multisection inputs between the two kernels.
 */
int figaro_sigma_bidiag(const double *R, int64_t n, int64_t ldr, double *sigma,
                        void *ws, size_t ws_bytes, void *stream);
/*
 * The squareroot-free route (Related Works: dqds, when only the singular values
 * are required): the bidiagonalisation of figaro_sigma_bidiag, then the
 * differential qd algorithm with shifts on the squared bidiagonal entries (one
 * thread: shifted transforms, bottom deflation, a zero-shift repeat of any
 * transform that would lose positivity).  Same arguments, workspace and n <= 128
 * as figaro_sigma_bidiag.
 */
int figaro_sigma_dqds(const double *R, int64_t n, int64_t ldr, double *sigma, void *ws, size_t ws_bytes,
                      void *stream);

/*
 * figaro_sigma without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  The workspace is a static array of the library
 * (256 bytes + 512 x 512 FP64 = 2 MiB + 256 bytes) of which every GPU holds its
 * own copy until the process ends; its address on the current device is looked
 * up on the first call there.  Same route, kernels and results as figaro_sigma;
 * no allocation and no stage timing.  `stream` must belong to the current
 * device.  Calls that overlap on one GPU race on the shared array.
 * FIGARO_EINVAL for n outside [1, 512] (sizes beyond the static array), NULL
 * pointers or ldr < n; FIGARO_EHIP if the array's address cannot be obtained.
 */
int figaro_sigma_noalloc(const double *R, int64_t n, int64_t ldr, double *sigma, void *stream);

/*
 * Synchronous: waits for `stream`, then reads the device status word left in
 * `ws` by the last figaro_r / figaro_compact / plan execution that used it.
 * *code receives FIGARO_OK, FIGARO_EUNSORTED or FIGARO_ETIMEOUT.
 */
int figaro_status(const void *ws, void *stream, int32_t *code);

/* Message of the last failure on the calling thread ("" if none). */
const char *figaro_last_error(void);

/*
 * Per-stage device timing, for measurement.  Off by default.  When on, every
 * kernel launch of the library is bracketed by two hipEventRecord calls on
 * its stream, under a stage name: "group", "scan_reduce", "scan_carry",
 * "scan_write", "assemble", a region tree ("tsqr_m1", "tsqr_m2", "tsqr_heads",
 * "tsqr_tails"), "tsqr_root", "sign", "refine_gram", "refine_solve",
 * "jacobi", "sigma_bidiag", "sigma_msect", "sigma_dqds"; a plan's stages
 * ("tsqr_narrow" for its narrow trees, "tsqr_np<w>", "root_np<w>",
 * "sigma_np<w>" per padded width w) and "plan_graph" for a graph launch.
 * figaro_timing_read is synchronous: it waits for the recorded events, writes
 * up to `cap` entries (stage name, total milliseconds, number of launches)
 * accumulated since the previous read, sets *count and clears the record.
 * Names are static strings owned by the library.
 */
int figaro_timing_enable(int32_t on);
int figaro_timing_read(const char **names, double *ms, int32_t *launches, int32_t cap,
                       int32_t *count);

/*
 * Singular values and right singular vectors of R (Abstract: the right
 * singular vectors of the join; Related Works: the SVD of the join through R):
 * one-sided Jacobi as in figaro_sigma_jacobi with every rotation also applied
 * to the columns of V, which starts as the identity, so that R V = U diag(sigma)
 * with V orthogonal.  R (device, n x n, ld ldr >= n) is read only.  sigma
 * (device, n) receives the values descending (equal values in column order);
 * V (device, n x n row-major, ld ldv >= n) column j receives the vector of
 * sigma[j] (unique up to sign where sigma[j] is simple).  FP64 throughout; the
 * right singular vectors of J equal those of R.  n <= 128.  Workspace:
 * figaro_svd_workspace_size(n) bytes, 256-byte aligned (a control block and V's
 * columns during the sweeps).  Asynchronous.
 */
int figaro_svd_workspace_size(int64_t n, size_t *bytes);
int figaro_svd(const double *R, int64_t n, int64_t ldr, double *sigma, double *V, int64_t ldv, void *ws,
               size_t ws_bytes, void *stream);

/* ------------------------------------------------------------ unsorted inputs, memory */

/*
 * The method takes relations sorted by the join attribute (Experiments
 * section).  figaro_sort_table lifts that precondition: it writes `in`'s rows
 * to `out` (device, same dtype and cols, row-major with ld_out >= cols) and
 * their keys to keys_out (device, rows entries) in ascending signed key order,
 * rows with equal keys in their input order (a stable sort; LSD radix sort of
 * the keys with their row indices, 8 passes of 4-bit digits, then a row
 * gather).  in->keys is required.  `out` must not alias in->data; keys_out may
 * alias in->keys only if the caller no longer needs the unsorted keys (they
 * are read in the first pass).  Workspace: figaro_sort_workspace_size(rows)
 * bytes, 256-byte aligned, caller-owned.  Asynchronous.
 */
int figaro_sort_workspace_size(int64_t rows, size_t *bytes);
int figaro_sort_table(const figaro_table *in, void *out, int64_t ld_out, int32_t *keys_out, void *ws,
                      size_t ws_bytes, void *stream);

/*
 * Memory footprint of the compact path against the materialised join (the
 * paper's memory claim, Abstract): the join's rows (sum m1_g m2_g), its bytes
 * in the inputs' element type (join_rows x (n1 + n2)), the inputs (rows and
 * keys), the compact matrix as stored by the form (rows and bytes), and the
 * workspace of figaro_r.  Synchronous: waits for `stream`, then reads the
 * counts that figaro_r or figaro_compact left in `ws` for these tables.
 */
typedef struct figaro_memory {
    int64_t groups, join_rows, compact_rows;
    double input_bytes, compact_bytes, workspace_bytes, join_bytes;
} figaro_memory;
int figaro_memory_report(const figaro_table *A, const figaro_table *B, int32_t precision, const void *ws,
                         size_t ws_bytes, void *stream, figaro_memory *out);

/* ------------------------------------------------------------ batching */

/*
 * A plan runs many independent two-table problems (of uneven sizes) in one
 * launch sequence, captured once in a HIP graph and replayed by
 * figaro_plan_execute.  Each instance is a Cartesian product or natural join
 * exactly as in figaro_r.  Outputs: R_i (FP64, N_i x N_i, row-major, packed
 * one after another at offsets given by figaro_plan_offsets) and sigma_i.
 */
typedef struct figaro_instance {
    figaro_table A, B;
} figaro_instance;

typedef struct figaro_plan figaro_plan;

/* Host-only; copies the instance descriptors (the data pointers must stay valid). */
int figaro_plan_create(const figaro_instance *inst, int32_t count, int32_t precision,
                       figaro_plan **out);
int figaro_plan_workspace_size(const figaro_plan *plan, size_t *bytes);
/* r_off[i], s_off[i] (host, count entries): element offsets of R_i and sigma_i; totals in *r_total, *s_total. */
int figaro_plan_offsets(const figaro_plan *plan, int64_t *r_off, int64_t *s_off,
                        int64_t *r_total, int64_t *s_total);
/*
 * Enqueue the whole batch on `stream`.  The batch runs stage by stage, each
 * stage one launch (or a short sequence) over every instance, driven by device
 * tables of per-instance descriptors:
 *   grouping (one launch for all Cartesian instances; a keyed instance runs its
 *   own grouping), head/tail scans (one tile-reduce / carry-scan / tile-write
 *   sequence over the tiles of every table), the regions' TSQR (one tree launch
 *   over the leaves of every region of padded width up to 64 of every instance,
 *   the widest leaves first, each region with its own node counters and root;
 *   wider regions per region),
 *   the roots (one launch per padded width for the Cartesian instances of the
 *   two-sided form; the others, and the refinement sweep, per instance), and
 *   sigma by the bidiagonal route of figaro_sigma_bidiag (two launches per width
 *   class over all instances, the classes side by side on the plan's side
 *   streams; the multisection there locates each value with 16 lanes and 16
 *   points per round, 14 rounds, or at width class 128 with 4 lanes and 4
 *   points per round, 24 rounds).  Without refinement, where the tuning table
 *   says so, the instances with n1 + n2 > 64 and the others run their trees,
 *   roots and sigma as two chains side by side instead (after the assembly).
 *   The side streams (four, default priority) are forked from `stream` by an
 *   event and joined back before the call's last launch.  Each instance owns one
 *   slice of `ws`; the multisection inputs sit after the slices.  Instances need
 *   n1 + n2 <= 128.
 * The first call on a plan creates its side streams and events (destroyed by
 * figaro_plan_destroy).  The first call with a given (ws, R, sigma) allocates
 * and uploads that triple's launch tables (synchronous; freed by
 * figaro_plan_destroy) and
 * captures the launch sequence into a HIP graph on a private stream; every call
 * (the first included) launches that graph on `stream`.  Later calls with the
 * same triple allocate nothing.  Calls that share `ws` must not overlap.
 */
int figaro_plan_execute(figaro_plan *plan, void *ws, size_t ws_bytes, double *R, double *sigma,
                        void *stream);
/*
 * The same launches as figaro_plan_execute, enqueued one by one on `stream`
 * without a graph (the launch tables of the triple are uploaded as there), so
 * that the stage timing of figaro_timing_enable records every stage.
 */
int figaro_plan_execute_eager(figaro_plan *plan, void *ws, size_t ws_bytes, double *R, double *sigma,
                              void *stream);
/*
 * Frees the plan, its graphs, launch tables, side streams and events.  A plan that
 * has executed first waits for the device (hipDeviceSynchronize), so that launches
 * of its graphs still in flight finish before their resources go; the autotuner
 * does the same before it drops the plan's graphs.
 */
void figaro_plan_destroy(figaro_plan *plan);

/* ------------------------------------------------------------ autotuning */

/*
 * The TSQR reduction of each region of padded width <= 128 runs one of two
 * tree kernels (one workgroup per leaf -- at width 128 the streaming panel
 * tree -- or one wave per leaf) with leaves of a chosen number of row blocks
 * and a chosen tree arity.  A process-wide tuning table, keyed by
 * (accumulation type, padded width, single call or plan, log2 of the rows),
 * holds the choice; its built-in defaults were measured on MI355X.  It also
 * holds each plan sigma class's route and whether plans run their two chains
 * side by side (set by hand or a cache file; the autotuner leaves it).
 *
 * figaro_plan_autotune / figaro_r_autotune time every candidate of the table
 * on the caller's own problem (the same buffers figaro_plan_execute / figaro_r
 * take: one warm-up and three timed runs per candidate, stage events on
 * `stream`), keep the fastest per class of regions, and set the table entries
 * of the row counts the problem holds.  A plan's classes are tuned alone, then
 * together on their shared launch.  The chaining mode is not tuned (the table
 * entry, default one chain after the other).  Synchronous; they allocate launch
 * tables, overwrite R / sigma / ws, drop the plan's captured graphs (the next
 * execution captures again), and record stage events into the timing of
 * figaro_timing_enable (consumed).  Workspace sizes do not depend on the
 * table.  Not thread-safe against concurrent calls that lay out regions.
 */
int figaro_plan_autotune(figaro_plan *plan, void *ws, size_t ws_bytes, double *R, double *sigma, void *stream);
int figaro_r_autotune(const figaro_table *A, const figaro_table *B, int32_t precision, double *R, int64_t ldr,
                      void *ws, size_t ws_bytes, void *stream);
/*
 * Tuning cache: JSON lines, one entry per line with the fields arch ("gfx950"),
 * acc_f64, np, batched, rows_log2, kind (0 workgroup tree, 1 wave tree),
 * leaf_blocks, arity, ms (acc_f64 2: a plan sigma class's route, kind 0
 * multisection, 1 dqds; acc_f64 3, np 1 for FP64 accumulation else 0: kind 1
 * plans run their chains side by side).  figaro_tune_load merges a file into
 * the table (the
 * file named by the environment variable FIGARO_TUNE_CACHE is merged at first
 * use); figaro_tune_save writes the whole table; figaro_tune_dump copies it into
 * buf (NUL-terminated, at most cap bytes) and its full length into *len.
 */
int figaro_tune_load(const char *path);
int figaro_tune_save(const char *path);
int figaro_tune_dump(char *buf, size_t cap, size_t *len);

#ifdef __cplusplus
}
#endif
#endif /* FIGARO_H */
