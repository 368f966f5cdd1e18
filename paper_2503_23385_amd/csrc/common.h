// Internal declarations shared by the host runtime and the kernels of the
// gfx950 Figaro library.  Nothing here is part of the public ABI (figaro.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace figaro {

// device status codes (mirror the public FIGARO_* codes)
constexpr int kStatusOk = 0;
constexpr int kStatusUnsorted = -2;
constexpr int kStatusTimeout = -5;

// counts[] slots: groups, region-1 rows (sum m1_g), region-2 rows (sum m2_g - 1),
// join rows, runs of A and B (scratch), a scratch slot, and sum (m1_g - 1).
enum : int {
    CNT_G = 0, CNT_R1 = 1, CNT_R2 = 2, CNT_JOIN = 3, CNT_UA = 4, CNT_UB = 5, CNT_TMP = 6,
    CNT_TA = 7, CNT_SLOTS = 8
};

// Device view of the group table (structure of arrays, ascending key order).
struct Groups {
    int32_t *key, *offA, *m1, *offB, *m2, *r1, *r2;
    int64_t *counts;  // CNT_* slots
};

// Which table a head/tail scan runs over: for group g its rows start at off[g],
// it has size[g] rows, the other table has other[g] rows (the tails are scaled by
// sqrt(other[g])), and tail i of the group goes to output row
// obase[g] - (sub_g ? g : 0) + i - 1.
struct ScanSide {
    const int32_t *off, *size, *other, *obase;
    int32_t sub_g;
};

// One source of rows for the TSQR: `rows` rows (device count if rows_dev != nullptr,
// else rows_host) of width `width`, placed at column `col_off` of the virtual row;
// ld in elements.
struct RowSrc {
    const void *p;
    const int64_t *rows_dev;
    int64_t rows_host;
    int64_t ld;
    int32_t col_off;
    int32_t width;
};

// Copies count elements through registers with U loads in flight: v = ld(e) for
// e = first, first + stride, ..., then st(e, v).  A plain loop whose body loads and
// then stores waits for every load in turn; here the U loads of a round are issued
// together.  ld is also called with e = count - 1 in place of indices past the end, so
// it must be safe (and is only used) for e < count.
template <int U, typename T, typename Ld, typename St>
__device__ inline void staged_copy(int count, int first, int stride, Ld ld, St st)
{
    for (int e0 = first; e0 < count; e0 += U * stride) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int e = e0 + u * stride;
            v[u] = ld(e < count ? e : count - 1);
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int e = e0 + u * stride;
            if (e < count) st(e, v[u]);
        }
    }
}

// Row r of the stacked sources (rows [0, rows0) of s0, then s1), column k of the virtual
// row.  r must be a row of the stacked sources; the source column is clamped into range,
// so the load is always valid and needs no branch.  stacked_real says whether the
// element is real (else it counts as 0); keeping that test out of the load lets a round
// of loads be issued together.
template <typename Tin, typename Tacc>
__device__ inline Tacc load_stacked(const RowSrc &s0, const RowSrc &s1, int64_t rows0, int64_t r, int k)
{
    const bool first = r < rows0;
    const Tin *p = (const Tin *)(first ? s0.p : s1.p);
    const int64_t lr = first ? r : r - rows0, ld = first ? s0.ld : s1.ld;
    const int off = first ? s0.col_off : s1.col_off, w = first ? s0.width : s1.width;
    const int c = k - off;
    return (Tacc)p[lr * ld + (c < 0 ? 0 : (c >= w ? w - 1 : c))];
}

__device__ inline bool stacked_real(const RowSrc &s0, const RowSrc &s1, int64_t rows0, int64_t r, int k)
{
    const bool first = r < rows0;
    const int c = k - (first ? s0.col_off : s1.col_off);
    return c >= 0 && c < (first ? s0.width : s1.width);
}

// Elements handled per block by the grouping kernels.
constexpr int kGroupBlock = 2048;
constexpr int kGroupThreads = 256;

// ---------------------------------------------------------------- launchers
// grouping (kernels_group.hip)
hipError_t launch_group_init(int32_t *status, int64_t *counts, int32_t *ticket, int32_t *flags,
                             int64_t nflags, hipStream_t s);
// Cartesian product: the initialisation of launch_group_init and the one-group table in one launch.
hipError_t launch_group_cartesian(int32_t *status, int32_t *flags, int64_t nflags, Groups g, int64_t m1,
                                  int64_t m2, hipStream_t s);
// The same for a batch of Cartesian products (device table, one entry per instance).
struct CartInit {
    int32_t *status;
    int32_t *flags;
    int64_t nflags;
    Groups g;
    int64_t m1, m2;
};
hipError_t launch_group_cartesian_batch(const CartInit *tab, int count, hipStream_t s);
hipError_t launch_group_keys(const int32_t *kA, int64_t m1, const int32_t *kB, int64_t m2,
                             Groups g, int32_t *blkA, int32_t *blkB, int32_t *runA, int32_t *runB,
                             int32_t *matchA, int32_t *blkM, int64_t *blkS, int32_t *status,
                             hipStream_t s);

// head/tail scans and assembly (kernels_scan.hip)
struct ScanPlan {
    int q;        // row groups per tile
    int rpt;      // rows per thread
    int cpt;      // columns per thread
    int tile_rows;
    int64_t ntiles;
};
ScanPlan scan_plan(int64_t m, int64_t n, int in_bytes);
// Three launches: tile reduce, carry scan, tile write (tileF: ntiles ints; tileS, carry:
// ntiles x n doubles of scratch).  heads[g] receives H(X_g) = (sum of the group's rows) / sqrt(size).
// One table's head/tail scan: its rows, output tails (out) and heads, and the tile scratch.
struct ScanJob {
    const void *in;
    int64_t ld;
    int32_t m, n, q;
    ScanSide side;
    void *out;
    double *heads;
    int32_t *tileF;
    double *tileS;
    double *carry;
    int64_t ntiles;
    Groups g;           // the group table the job's side arrays belong to
    int32_t cartesian;  // one group spanning the whole table
};
ScanJob scan_job(const void *X, int64_t ldx, int64_t m, int64_t n, ScanSide side, void *out, double *heads,
                 int32_t *tileF, double *tileS, double *carry, const ScanPlan &sp);
// Scans one or two jobs (an empty second job has ntiles = 0) in three launches (tile
// reduce, carry scan, tile write; pass 0, 1 or 2 alone, or all three for pass < 0); two
// jobs need the same cpt and storage types.
hipError_t launch_seg_scan(const ScanJob &j0, const ScanJob &j1, int cpt, int in_f64, int out_f64, Groups g,
                           int cartesian, hipStream_t s, int pass = -1);
// One pass (0 tile reduce, 1 carry scan, 2 tile write) over a batch of jobs (device table
// `jobs`, each with its own group table): tile_map[b] = (job, tile) for each of the ntiles
// tile blocks, col_map[b] = (job, first of 64 columns) for each of the ncols carry blocks; every job of
// the batch has the same cpt and the same input and storage types.
hipError_t launch_seg_scan_batch(int pass, const ScanJob *jobs, const int2 *tile_map, int64_t ntiles,
                                 const int2 *col_map, int64_t ncols, int cpt, int in_f64, int out_f64, hipStream_t s);
// Claim 1 region 1: [sqrt(m2_g) A_r | H(B_g)].
hipError_t launch_assemble_a(const void *A, int in_f64, int64_t lda, int64_t m1, int64_t n1,
                             int64_t n2, Groups g, int cartesian, const double *heads, void *M1,
                             int out_f64, hipStream_t s);
// Head rows of the two-sided form: row g = [sqrt(m2_g) H(A_g) | sqrt(m1_g) H(B_g)].
hipError_t launch_head_rows(Groups g, int64_t gcap, const double *headsA, const double *headsB,
                            int64_t n1, int64_t n2, void *out, int out_f64, hipStream_t s);

// TSQR (kernels_tsqr.hip)
int tsqr_padded_width(int n);               // padded template width for n, 0 if unsupported
int tsqr_block_rows(int np, int acc_f64);   // rows per streamed block for padded width np
int tsqr_panel_rows(int np, int acc_f64);   // rows per block of the panel kernel (np 128..512)
// Blocked panel kernel for padded widths 128, 256, 512 (same contract as launch_tsqr_stream).
hipError_t launch_tsqr_panel(int np, int acc_f64, int in_f64, const double *init, int64_t init_ld, RowSrc s0,
                             RowSrc s1, int nsrc, int width, int tri_rows, int nwg, double *tri, int64_t tri_stride,
                             hipStream_t s);
// Arity of the in-kernel tree for a region of `width` columns at padded width np: one
// block of rows holds arity - 1 sibling triangles.
int tsqr_tree_arity(int np, int width);
// Slots (triangles) and counters needed by the in-kernel tree over nleaves leaves.
void tsqr_tree_sizes(int nleaves, int arity, int64_t *slots, int64_t *counters);
// Reduce the rows of s0 (then s1) into nwg triangles of `width` rows x np columns (FP64),
// triangle b at tri + b * tri_stride, each starting from `init` (a triangle, ld init_ld)
// when init != nullptr, else from zero.  tri_rows > 0: the sources are stacks of triangles
// of that many rows (lets a block skip known-zero leading columns).
hipError_t launch_tsqr_stream(int np, int acc_f64, int in_f64, const double *init, int64_t init_ld,
                              RowSrc s0, RowSrc s1, int nsrc, int width, int tri_rows, int nwg,
                              double *tri, int64_t tri_stride, hipStream_t s);
// One region for the in-kernel tree: nleaves wave-level leaves over src, then a tree of
// the given arity whose nodes live in `slots` (width x np FP64 each) and whose per-node
// counters (zero on entry) live in `counters`; the region's triangle lands in root.
struct TreeRegion {
    RowSrc src;
    int32_t width, nleaves, arity;  // nleaves: the most leaves (slots and counters are sized for it)
    int64_t rows_per_leaf;          // leaves used = min(nleaves, ceil(rows / rows_per_leaf)), at least 1
    double *slots;
    int32_t *counters;
    double *root;
    void *vbuf;  // wide regions: one reflector side buffer (wqr_vbuf_bytes) per leaf
};
// Wide regions (padded width 128, 256 or 512), one or two of the same width per launch:
// one workgroup per leaf of at most wqr_leaf_rows rows, each factorised in place by the
// blocked Householder QR; leaves' triangles merged pairwise up an in-kernel binary tree
// (slots and counters as tsqr_panel_tree_sizes).  in_f64: the regions' storage type.
hipError_t launch_wqr_tree(int np, int in_f64, const TreeRegion *regs, int nreg, hipStream_t s);
int64_t wqr_leaf_rows(int in_f64);
int64_t wqr_vbuf_bytes();
// top <- R of [top; bottom] for two FP64 upper triangles of width <= 512 (bottom is
// overwritten; vbuf: wqr_vbuf_bytes).  One workgroup.
hipError_t launch_wqr_merge(double *top, int64_t ld1, double *bottom, int64_t ld2, int width, double *vbuf,
                            hipStream_t s);
// dst (n x n) <- the w x w triangle src at rows [0, w), columns [off, off + w); zeros elsewhere.
hipError_t launch_wqr_pad(const double *src, int64_t lds, int w, int off, double *dst, int64_t ldd, int n,
                          hipStream_t s);
// One launch for one or two regions of the same padded width np (np <= 64), one workgroup
// per leaf, or one wave per leaf when wave_tree is set.
hipError_t launch_tsqr_tree(int np, int acc_f64, int in_f64, const TreeRegion *regs, int nreg,
                            hipStream_t s, int wave_tree = 0);
// One or two regions of padded width np <= 64 by Givens rotations (one wave per leaf, rows
// absorbed one at a time; FP64), tree nodes as in the wave tree.
hipError_t launch_givens_tree(int np, int in_f64, const TreeRegion *regs, int nreg, hipStream_t s);
// A batch of regions of padded width np <= 64 in one launch: device table regs, and
// map[i] = (region, leaf) for each of the nitems leaves (leaves beyond what a region's
// device-side row count needs exit at once).  wave_tree: one wave per leaf (triangles
// and tree nodes of the wave tree: rows per leaf a multiple of tsqr_wave_block_rows);
// else one workgroup per leaf (the workgroup tree of launch_tsqr_tree).
hipError_t launch_tsqr_tree_batch(int wave_tree, int np, int acc_f64, int in_f64, const TreeRegion *regs,
                                  const int2 *map, int64_t nitems, hipStream_t s);
// The wave-tree regions of every narrow width of a batch in one launch: item i is leaf
// map[i].y of region map[i].x of padded width map[i].z (4 .. 64).
hipError_t launch_tsqr_wtree_multi(int acc_f64, int in_f64, const TreeRegion *regs, const int4 *map, int64_t nitems,
                                   hipStream_t s);
int tsqr_wave_block_rows(int np);  // rows per block of the wave tree (np <= 64)
// Root of the two-sided form of a Cartesian product (N = na + nb <= 128): diag(R_TA, R_TB)
// absorbs the head row built from the head sums hA, hB; R (ld ldr) receives the result
// with row signs normalised.
hipError_t launch_merge_cartesian(int np, const double *Ta, int64_t lda, int na, const double *Tb, int64_t ldb, int nb,
                                  Groups g, const double *hA, const double *hB, double *R, int64_t ldr,
                                  hipStream_t s);
// The same for a batch of instances: one entry per instance, all of padded width np.
struct CartRoot {
    const double *Ta;
    int64_t lda;
    int32_t na;
    const double *Tb;
    int64_t ldb;
    int32_t nb;
    Groups g;
    const double *hA, *hB;
    double *R;
    int64_t ldr;
};
hipError_t launch_merge_cartesian_batch(int np, const CartRoot *tab, int count, hipStream_t s);
// out (na + nb rows, ld ldo) <- the upper triangular block diagonal [Ta 0; 0 Tb].
hipError_t launch_block_diag(const double *Ta, int64_t lda, int na, const double *Tb, int64_t ldb, int nb,
                             double *out, int64_t ldo, hipStream_t s);
// Wide regions of padded width 128 (one or two per launch): in-kernel binary tree over
// leaves that stream blocks of rows through LDS (kernels_panel.hip); wider regions take
// launch_wqr_tree.
hipError_t launch_tsqr_panel_tree(int np, int acc_f64, int in_f64, const TreeRegion *regs, int nreg, hipStream_t s);
// Node triangles and counters of a binary in-kernel tree over nleaves leaves (wide regions).
void tsqr_panel_tree_sizes(int nleaves, int64_t *slots, int64_t *counters);
hipError_t launch_sign_normalise(const void *Rin, int in_f64, int64_t ldin, int n, double *R,
                                 int64_t ldr, hipStream_t s);

// One FP64 refinement sweep (kernels_refine.hip; part 0: the Gram matrix only, 1: the rest,
// 2: both): from the approximate R~ (Rt, upper,
// positive diagonal) and the exact per-group Gram matrix of the join, R = chol(X)^T R~ with
// X = R~^-T (J^T J) R~^-1.  hB: the groups' heads of B (H(B_g), gcap x n2).  Scratch: gram
// and Y (N x N each), partial (partial_cap doubles, at least refine_partial_elems), failed
// (one int: 1 when X was not positive definite, then R = R~).
int64_t refine_partial_elems(int64_t n1, int64_t n2);
// One block of the closed-form Gram matrix (A^T A weighted, B^T B weighted, or the cross
// block), reduced over row chunks into per-chunk partials and then summed in a fixed order.
struct GramJob {
    const void *X;
    int64_t ld;
    int32_t m, nx, ny, mode, in_f64;
    const int32_t *off, *size, *other;
    const int64_t *Gp;
    int32_t cartesian;
    const double *hA, *hB;  // group heads H(A_g) (mode 2 only) and H(B_g)
    int32_t gx, gy, nch;
    int64_t rows_per_chunk;
    double *partial;
    double *gram;
    int32_t ldg, row0, col0, mirror;
};
// The three Gram jobs of one problem (partial: refine_partial_elems doubles); returns 3.
// With the heads of A (hA, gcap x n1; the two-sided form) the cross block is summed over
// the groups' heads (mode 2) instead of A's rows (mode 1).
int gram_jobs(const void *A, int in_f64, int64_t lda, int64_t m1, int n1, const void *B, int64_t ldb, int64_t m2,
              int n2, Groups g, int cartesian, const double *hA, const double *hB, int64_t gcap, double *partial,
              double *gram, GramJob *jobs, int64_t blocks);  // blocks: workgroups per job to aim at (<= 1024)
// A batch of Gram jobs of one input type: tile_map[b] = (job, ti, tj, chunk), red_map[b] =
// (job, block of 256 entries).
hipError_t launch_gram_batch(int in_f64, const GramJob *jobs, const int4 *tile_map, int64_t ntiles,
                             const int2 *red_map, int64_t nred, hipStream_t s);
// The N x N part of the sweep (N <= 128) for a batch of instances, one workgroup each
// (after their Gram matrices are formed).
struct RefineSmall {
    const double *gram, *Rt;
    int32_t ldt, n;
    double *Y;
    int32_t *failed;
    double *R;
    int64_t ldr;
};
hipError_t launch_refine_small_batch(const RefineSmall *tab, int count, hipStream_t s);
hipError_t launch_refine(const void *A, int in_f64, int64_t lda, int64_t m1, int n1, const void *B,
                         int64_t ldb, int64_t m2, int n2, Groups g, int cartesian, const double *hA,
                         const double *hB, int64_t gcap,
                         const double *Rt, int ldt, double *gram, double *Y, double *partial,
                         int64_t partial_cap, int32_t *failed, double *R, int64_t ldr, hipStream_t s,
                         int part = 2);

// Stable sort of a table's rows by key (kernels_sort.hip): out rows (ld_out) and keys_out
// in ascending signed key order, equal keys in input order.  ws: sort_workspace_bytes(n).
int64_t sort_workspace_bytes(int64_t n);
hipError_t launch_sort_table(const void *X, int elem_bytes, int64_t ld, int64_t n, int64_t cols, const int32_t *keys,
                             void *out, int64_t ld_out, int32_t *keys_out, void *ws, hipStream_t s);

// Jacobi (kernels_jacobi.hip)
// ctrl: 8 ints (ctrl[0] receives the sweep count, -1 after a timed-out run); scratch:
// jacobi_scratch_doubles(n) doubles (none for n <= 128).
int64_t jacobi_scratch_doubles(int n);
hipError_t launch_jacobi(const double *R, int n, int64_t ldr, double *sigma, int max_sweeps,
                         int32_t *ctrl, double *scratch, hipStream_t s);
// Singular values and right singular vectors of R (n <= 128): one-sided Jacobi that also
// rotates V (scratch: svd_v_scratch_doubles(n), V's columns during the sweeps); V (n x n,
// ld ldv) row i, column k = component i of the k-th right singular vector (sigma descending).
int64_t svd_v_scratch_doubles(int n);
hipError_t launch_svd_v(const double *R, int n, int64_t ldr, double *sigma, double *V, int64_t ldv, int max_sweeps,
                        int32_t *ctrl, double *scratch, hipStream_t s);
// The bidiagonal route for n <= 128: bidiagonalisation + multisection (ctrl[0] = 0 sweeps).
int64_t sigma_bidiag_scratch_doubles(int n);  // multisection inputs of the bidiagonal route (n <= 128)
// bidiagonalisation of R (one workgroup), leaving the multisection inputs in msin
hipError_t launch_sigma_bidiag(const double *R, int n, int64_t ldr, int32_t *ctrl, double *msin, hipStream_t s);
// multisection: one workgroup per singular value
hipError_t launch_sigma_msect(const double *msin, int n, double *sigma, hipStream_t s);
// dqds on the same inputs (the squared bidiagonal entries), one thread
hipError_t launch_sigma_dqds(const double *msin, int n, double *sigma, hipStream_t s);
// Width class (padded n: 8..128) of the bidiagonal route; 0 above 128.
int sigma_width_class(int n);
// Independent problems of one width class by the bidiagonal route, two launches; tab
// (device): 4 int64 per problem (element offset of its R in R, of its sigma in sigma, n,
// of its 2n + 2 multisection doubles in msin), R packed n x n (ld n).
hipError_t launch_sigma_batch(int npc, const double *R, double *sigma, const int64_t *tab, int count, double *msin,
                              hipStream_t s, int dqds = 0);  // dqds: the values by dqds, else by multisection

}  // namespace figaro
