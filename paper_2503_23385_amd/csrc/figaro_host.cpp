// Host runtime of the gfx950 Figaro library: argument checks, workspace
// layout, and the launch sequence behind the C ABI of include/figaro.h.
//
// The pipeline follows the paper's Figaro-GPU steps (Experiments section):
// heads and tails per key group, the compact matrix of Claim 1, a Householder
// QR of that matrix for R, and the singular values of R.  How each step runs
// on the device differs: segmented scans instead of one thread per column,
// no row/column-major transpose, and TSQR reductions instead of a library QR.
//
// The rows to be reduced are organised in regions, each reduced by its own
// TSQR to one triangle; the triangles are then merged into R:
//   Claim 1 form:   M1 = [sqrt(m2_g) A_r | H(B_g)] (width N) and
//                   M2 = [0 | sqrt(m1_g) T(B_g)]   (width n2 at column n1);
//   two-sided form: the same matrix with each group's M1 rows also replaced by
//                   their head and tail (the faster variant noted after Claim 1):
//                   heads [sqrt(m2_g) H(A_g) | sqrt(m1_g) H(B_g)] (width N),
//                   [sqrt(m2_g) T(A_g) | 0] (width n1) and M2 as above.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "common.h"
#include "../../include/figaro.h"

using namespace figaro;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char *where)
{
    return fail(FIGARO_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

// ------------------------------------------------------------ stage timing
//
// Process-wide record of stage events, guarded by a mutex: library calls may run on
// several host threads.  A thread that is capturing a graph records no events (events
// recorded into a capture would not measure replays).

struct TimingRec {
    const char *name;
    hipEvent_t a, b;
};

struct Timing {
    std::atomic<bool> on{false};
    std::mutex mu;
    std::vector<TimingRec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t get()  // caller holds mu
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};

Timing g_timing;
thread_local bool t_capturing = false;

// Brackets the launches of one stage with events when timing is on.
struct Stage {
    const char *name;
    hipStream_t s;
    hipEvent_t a = nullptr;
    Stage(const char *n, hipStream_t st) : name(n), s(st)
    {
        if (n && g_timing.on.load() && !t_capturing) {
            {
                std::lock_guard<std::mutex> lk(g_timing.mu);
                a = g_timing.get();
            }
            if (a) (void)hipEventRecord(a, s);
        }
    }
    ~Stage()
    {
        if (!a) return;
        std::lock_guard<std::mutex> lk(g_timing.mu);
        hipEvent_t b = g_timing.get();
        if (b) {
            (void)hipEventRecord(b, s);
            g_timing.recs.push_back({name, a, b});
        } else {
            g_timing.pool.push_back(a);
        }
    }
};

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

constexpr int kPrecMask = 0xff;
constexpr int kMaxTreeLeaves = 2048;
constexpr int64_t kLeafTarget = 256;
constexpr int kMaxPanelLeaves = 128;
constexpr int kPlanLanes = 8;  // parallel branches of a batched plan's graph

struct Shape {
    int64_t m1, n1, lda, m2, n2, ldb;
    int in_f64;
    bool keyed;
    int precision;  // FIGARO_PLAIN_FP64 / FIGARO_MIXED_FP32 / FIGARO_MIXED_FP32_REFINE
    bool two_sided;
    int64_t N() const { return n1 + n2; }
};

// A region: rows (device count in counts[cnt]) of `width` columns at column col_off,
// stored at `buf` (storage type of the form), reduced to one triangle at `root`.
struct Region {
    const char *name;
    size_t buf;
    int64_t rows_cap;
    int cnt;
    int width, col_off, np;
    bool wave;                // narrow tree kernel (np <= 64); else the panel tree kernel
    bool skip;                // rows absorbed directly by the root merge (no tree of its own)
    int leaves, arity;        // most leaves; tree arity
    int64_t rows_per_leaf;    // leaves follow the device row count: ceil(rows / rows_per_leaf)
    size_t slots, counters, root;
    int64_t ncounters;
};

struct Layout {
    size_t status, counts;
    size_t blkA, blkB, runA, runB, matchA, blkM, blkS;
    size_t g[7];
    int64_t gcap;
    size_t headsA, headsB;
    size_t tileF[2], tileS[2], carry[2];
    ScanPlan spA, spB;
    int m_f64;
    std::vector<Region> regions;
    size_t counters_base;
    int64_t counters_total;
    size_t rtmp[2];
    // refinement sweep (FIGARO_MIXED_FP32_REFINE only)
    bool refine;
    size_t rt, gram, gy, partial, failed;
    int64_t partial_cap;
    int np_root;
    size_t total;
    int nbA, nbB;
};

int check_table(const figaro_table *t, const char *name)
{
    if (!t) return fail(FIGARO_EINVAL, std::string(name) + " is NULL");
    if (t->rows < 0 || t->cols < 1) return fail(FIGARO_EINVAL, std::string(name) + ": rows < 0 or cols < 1");
    if (t->rows > INT32_MAX - 1) return fail(FIGARO_EINVAL, std::string(name) + ": more than 2^31-2 rows");
    if (t->ld < t->cols) return fail(FIGARO_EINVAL, std::string(name) + ": ld < cols");
    if (t->dtype != FIGARO_F32 && t->dtype != FIGARO_F64) return fail(FIGARO_EINVAL, std::string(name) + ": bad dtype");
    if (t->rows > 0 && !t->data) return fail(FIGARO_EINVAL, std::string(name) + ": data is NULL");
    return FIGARO_OK;
}

int make_shape(const figaro_table *A, const figaro_table *B, int32_t precision, Shape *sh)
{
    int rc = check_table(A, "A");
    if (rc) return rc;
    rc = check_table(B, "B");
    if (rc) return rc;
    if (A->dtype != B->dtype) return fail(FIGARO_EINVAL, "A and B must share a dtype");
    if ((A->keys == nullptr) != (B->keys == nullptr))
        return fail(FIGARO_EINVAL, "keys must be given for both tables or for neither");
    const int prec = precision & kPrecMask;
    if ((precision & ~(kPrecMask | FIGARO_TWO_SIDED)) != 0 ||
        (prec != FIGARO_PLAIN_FP64 && prec != FIGARO_MIXED_FP32 && prec != FIGARO_MIXED_FP32_REFINE))
        return fail(FIGARO_EINVAL, "unknown precision or flag");
    const int64_t N = A->cols + B->cols;
    if (N > FIGARO_MAX_N) return fail(FIGARO_EINVAL, "n1 + n2 exceeds FIGARO_MAX_N");
    if (tsqr_padded_width((int)N) == 0) return fail(FIGARO_EINVAL, "n1 + n2 wider than the TSQR kernels support");
    sh->m1 = A->rows;
    sh->n1 = A->cols;
    sh->lda = A->ld;
    sh->m2 = B->rows;
    sh->n2 = B->cols;
    sh->ldb = B->ld;
    sh->in_f64 = A->dtype == FIGARO_F64;
    sh->keyed = A->keys != nullptr;
    sh->precision = prec;
    sh->two_sided = (precision & FIGARO_TWO_SIDED) != 0;
    return FIGARO_OK;
}

int env_int(const char *name, int dflt)
{
    const char *v = std::getenv(name);
    if (!v || !*v) return dflt;
    const int x = std::atoi(v);
    return x > 0 ? x : dflt;
}

Region make_region(const char *name, int64_t rows_cap, int cnt, int width, int col_off, int acc_f64)
{
    Region r;
    r.name = name;
    r.rows_cap = std::max<int64_t>(0, rows_cap);
    r.cnt = cnt;
    r.width = width;
    r.col_off = col_off;
    r.np = tsqr_padded_width(width);
    r.wave = r.np <= 64;
    const int br = tsqr_block_rows(r.np, acc_f64);
    // Leaf sizes (fixed through FIGARO_LEAF_BLOCKS / FIGARO_WG_LEAF_BLOCKS).  Narrow trees
    // (measured): leaves of two blocks, lengthened to keep a region at kLeafTarget leaves
    // (two per compute unit when the two tails share a launch): shorter leaves add
    // workgroups that wait for a compute unit, longer ones add sequential column steps.
    // The wide tree keeps at most one leaf per compute unit and a half.
    static const int wave_blocks = env_int("FIGARO_LEAF_BLOCKS", 0);
    static const int wg_blocks = env_int("FIGARO_WG_LEAF_BLOCKS", 4);
    if (!r.wave) {
        r.rows_per_leaf = (int64_t)wg_blocks * br;
    } else if (wave_blocks > 0) {
        r.rows_per_leaf = (int64_t)wave_blocks * br;
    } else {
        const int64_t per_leaf = (r.rows_cap + kLeafTarget - 1) / kLeafTarget;
        r.rows_per_leaf = std::max<int64_t>(2 * br, (per_leaf + br - 1) / br * br);
    }
    const int64_t leaves = (r.rows_cap + r.rows_per_leaf - 1) / r.rows_per_leaf;
    r.leaves = (int)std::max<int64_t>(1, std::min<int64_t>(leaves, r.wave ? kMaxTreeLeaves : kMaxPanelLeaves));
    r.ncounters = 0;
    r.skip = false;
    r.arity = r.wave ? tsqr_tree_arity(r.np, width) : 2;
    return r;
}

Layout make_layout(const Shape &s)
{
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 1));
        return o;
    };
    L.status = take(sizeof(int32_t) * 4);
    L.counts = take(sizeof(int64_t) * CNT_SLOTS);
    L.nbA = (int)((s.m1 + kGroupBlock - 1) / kGroupBlock);
    L.nbB = (int)((s.m2 + kGroupBlock - 1) / kGroupBlock);
    if (s.keyed) {
        L.blkA = take(sizeof(int32_t) * (L.nbA + 1));
        L.blkB = take(sizeof(int32_t) * (L.nbB + 1));
        L.runA = take(sizeof(int32_t) * (s.m1 + 1));
        L.runB = take(sizeof(int32_t) * (s.m2 + 1));
        L.matchA = take(sizeof(int32_t) * (s.m1 + 1));
        L.blkM = take(sizeof(int32_t) * (L.nbA + 1));
        L.blkS = take(sizeof(int64_t) * 3 * (L.nbA + 1));
        L.gcap = std::max<int64_t>(1, std::min(s.m1, s.m2));
    } else {
        L.blkA = L.blkB = L.runA = L.runB = L.matchA = L.blkM = L.blkS = 0;
        L.gcap = 1;
    }
    for (int i = 0; i < 7; i++) L.g[i] = take(sizeof(int32_t) * L.gcap);
    L.headsB = take(sizeof(double) * L.gcap * s.n2);
    L.headsA = s.two_sided ? take(sizeof(double) * L.gcap * s.n1) : 0;
    L.m_f64 = s.precision == FIGARO_PLAIN_FP64;
    const size_t esz = L.m_f64 ? 8 : 4;
    L.spB = scan_plan(s.m2, s.n2, s.in_f64 ? 8 : 4);
    L.tileF[1] = take(sizeof(int32_t) * std::max<int64_t>(1, L.spB.ntiles));
    L.tileS[1] = take(sizeof(double) * std::max<int64_t>(1, L.spB.ntiles) * s.n2);
    L.carry[1] = take(sizeof(double) * std::max<int64_t>(1, L.spB.ntiles) * s.n2);
    if (s.two_sided) {
        L.spA = scan_plan(s.m1, s.n1, s.in_f64 ? 8 : 4);
        L.tileF[0] = take(sizeof(int32_t) * std::max<int64_t>(1, L.spA.ntiles));
        L.tileS[0] = take(sizeof(double) * std::max<int64_t>(1, L.spA.ntiles) * s.n1);
        L.carry[0] = take(sizeof(double) * std::max<int64_t>(1, L.spA.ntiles) * s.n1);
    } else {
        L.spA = ScanPlan{};
        L.tileF[0] = L.tileS[0] = L.carry[0] = 0;
    }
    const int N = (int)s.N();
    if (!s.two_sided) {
        Region a = make_region("tsqr_m1", s.m1, CNT_R1, N, 0, L.m_f64);
        Region b = make_region("tsqr_m2", s.m2 - 1, CNT_R2, (int)s.n2, (int)s.n1, L.m_f64);
        a.buf = take(esz * std::max<int64_t>(1, a.rows_cap) * N);
        b.buf = take(esz * std::max<int64_t>(1, b.rows_cap) * s.n2);
        L.regions = {a, b};
    } else {
        Region h = make_region("tsqr_heads", L.gcap, CNT_G, N, 0, L.m_f64);
        // Cartesian product: a single head row, absorbed by the root merge itself.
        h.skip = !s.keyed;
        Region ta = make_region("tsqr_ta", s.m1 - 1, CNT_TA, (int)s.n1, 0, L.m_f64);
        Region tb = make_region("tsqr_tb", s.m2 - 1, CNT_R2, (int)s.n2, (int)s.n1, L.m_f64);
        h.buf = take(esz * h.rows_cap * N);
        ta.buf = take(esz * std::max<int64_t>(1, ta.rows_cap) * s.n1);
        tb.buf = take(esz * std::max<int64_t>(1, tb.rows_cap) * s.n2);
        L.regions = {h, ta, tb};
    }
    int64_t ctot = 0;
    for (Region &r : L.regions) {
        const size_t tsz = sizeof(double) * (size_t)r.width * r.np;
        int64_t ns = 0, nc = 0;
        if (r.wave) tsqr_tree_sizes(r.leaves, r.arity, &ns, &nc);
        else tsqr_panel_tree_sizes(r.leaves, &ns, &nc);
        r.slots = take(tsz * ns);
        r.ncounters = nc;
        r.counters = (size_t)ctot;  // index into the shared counter block
        ctot += nc;
        r.root = take(tsz);
    }
    L.counters_total = ctot;
    L.counters_base = take(sizeof(int32_t) * std::max<int64_t>(1, ctot));
    L.np_root = tsqr_padded_width(N);
    L.rtmp[0] = take(sizeof(double) * N * L.np_root);
    L.rtmp[1] = take(sizeof(double) * N * L.np_root);
    L.refine = s.precision == FIGARO_MIXED_FP32_REFINE;
    if (L.refine) {
        L.rt = take(sizeof(double) * N * N);
        L.gram = take(sizeof(double) * N * N);
        L.gy = take(sizeof(double) * N * N);
        L.partial_cap = refine_partial_elems(s.n1, s.n2);
        L.partial = take(sizeof(double) * L.partial_cap);
        L.failed = take(sizeof(int32_t));
    } else {
        L.rt = L.gram = L.gy = L.partial = L.failed = 0;
        L.partial_cap = 0;
    }
    L.total = off;
    return L;
}

template <typename T>
T *at(void *ws, size_t off) { return (T *)((char *)ws + off); }

Groups groups_of(void *ws, const Layout &L)
{
    Groups g;
    g.key = at<int32_t>(ws, L.g[0]);
    g.offA = at<int32_t>(ws, L.g[1]);
    g.m1 = at<int32_t>(ws, L.g[2]);
    g.offB = at<int32_t>(ws, L.g[3]);
    g.m2 = at<int32_t>(ws, L.g[4]);
    g.r1 = at<int32_t>(ws, L.g[5]);
    g.r2 = at<int32_t>(ws, L.g[6]);
    g.counts = at<int64_t>(ws, L.counts);
    return g;
}

int check_ws(const Layout &L, void *ws, size_t ws_bytes)
{
    if (!ws) return fail(FIGARO_EINVAL, "workspace is NULL");
    if (((uintptr_t)ws) % kAlign) return fail(FIGARO_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total)
        return fail(FIGARO_EWORKSPACE, "workspace too small: need " + std::to_string(L.total) + " bytes");
    return FIGARO_OK;
}

#define HIPCHK(expr, where)                               \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

// Grouping, head/tail scans and assembly: fills the regions' row buffers (the head rows
// of the two-sided form only when head_rows is set).
int run_compact(const figaro_table *A, const figaro_table *B, const Shape &sh, const Layout &L,
                void *ws, hipStream_t s, bool head_rows = true)
{
    Groups g = groups_of(ws, L);
    int32_t *status = at<int32_t>(ws, L.status);
    {
        Stage st("group", s);
        if (sh.keyed) {
            HIPCHK(launch_group_init(status, g.counts, nullptr, at<int32_t>(ws, L.counters_base),
                                     L.counters_total, s),
                   "init");
            HIPCHK(launch_group_keys(A->keys, sh.m1, B->keys, sh.m2, g, at<int32_t>(ws, L.blkA),
                                     at<int32_t>(ws, L.blkB), at<int32_t>(ws, L.runA),
                                     at<int32_t>(ws, L.runB), at<int32_t>(ws, L.matchA),
                                     at<int32_t>(ws, L.blkM), at<int64_t>(ws, L.blkS), status, s),
                   "grouping");
        } else {
            HIPCHK(launch_group_cartesian(status, at<int32_t>(ws, L.counters_base), L.counters_total, g, sh.m1,
                                          sh.m2, s),
                   "grouping");
        }
    }
    double *hB = at<double>(ws, L.headsB);
    const Region &rb = L.regions.back();  // region of B's tails in both forms
    const ScanJob none{};
    ScanSide sideB{g.offB, g.m2, g.m1, g.r2, 0};
    const ScanJob jb = scan_job(B->data, sh.ldb, sh.m2, sh.n2, sideB, at<void>(ws, rb.buf), hB,
                                at<int32_t>(ws, L.tileF[1]), at<double>(ws, L.tileS[1]),
                                at<double>(ws, L.carry[1]), L.spB);
    if (!sh.two_sided) {
        {
            Stage st("scan", s);
            HIPCHK(launch_seg_scan(jb, none, L.spB.cpt, sh.in_f64, L.m_f64, g, !sh.keyed, s),
                   "head/tail scan of B");
        }
        Stage st("assemble", s);
        HIPCHK(launch_assemble_a(A->data, sh.in_f64, sh.lda, sh.m1, sh.n1, sh.n2, g, !sh.keyed, hB,
                                 at<void>(ws, L.regions[0].buf), L.m_f64, s),
               "region-1 assembly");
    } else {
        double *hA = at<double>(ws, L.headsA);
        ScanSide sideA{g.offA, g.m1, g.m2, g.r1, 1};
        const ScanJob ja = scan_job(A->data, sh.lda, sh.m1, sh.n1, sideA, at<void>(ws, L.regions[1].buf), hA,
                                    at<int32_t>(ws, L.tileF[0]), at<double>(ws, L.tileS[0]),
                                    at<double>(ws, L.carry[0]), L.spA);
        {
            // both tables in one launch per pass when their tiles have the same column layout
            Stage st("scan", s);
            if (L.spA.cpt == L.spB.cpt) {
                HIPCHK(launch_seg_scan(jb, ja, L.spB.cpt, sh.in_f64, L.m_f64, g, !sh.keyed, s),
                       "head/tail scans");
            } else {
                HIPCHK(launch_seg_scan(jb, none, L.spB.cpt, sh.in_f64, L.m_f64, g, !sh.keyed, s),
                       "head/tail scan of B");
                HIPCHK(launch_seg_scan(ja, none, L.spA.cpt, sh.in_f64, L.m_f64, g, !sh.keyed, s),
                       "head/tail scan of A");
            }
        }
        if (head_rows) {
            Stage st("assemble", s);
            HIPCHK(launch_head_rows(g, L.gcap, hA, hB, sh.n1, sh.n2, at<void>(ws, L.regions[0].buf),
                                    L.m_f64, s),
                   "head rows");
        }
    }
    return FIGARO_OK;
}

TreeRegion tree_region(const Region &r, const Layout &L, void *ws)
{
    Groups g = groups_of(ws, L);
    TreeRegion t;
    t.src = RowSrc{at<void>(ws, r.buf), g.counts + r.cnt, 0, r.width, 0, r.width};
    t.width = r.width;
    t.nleaves = r.leaves;
    t.arity = r.arity;
    t.rows_per_leaf = r.rows_per_leaf;
    t.slots = at<double>(ws, r.slots);
    t.counters = at<int32_t>(ws, L.counters_base) + r.counters;
    t.root = at<double>(ws, r.root);
    return t;
}

// All regions, each by its in-kernel tree; regions of equal padded width share a launch.
int run_regions(const Layout &L, int acc_f64, void *ws, hipStream_t s)
{
    const size_t nr = L.regions.size();
    std::vector<bool> done(nr, false);
    for (size_t i = 0; i < nr; i++) {
        if (done[i]) continue;
        const Region &r = L.regions[i];
        done[i] = true;
        if (r.skip) continue;
        TreeRegion tr[2] = {tree_region(r, L, ws), TreeRegion{}};
        int n = 1;
        const char *name = r.name;
        for (size_t j = i + 1; j < nr && n < 2; j++) {
            if (!done[j] && !L.regions[j].skip && L.regions[j].np == r.np) {
                tr[n++] = tree_region(L.regions[j], L, ws);
                done[j] = true;
                name = "tsqr_tails";
            }
        }
        Stage st(name, s);
        if (r.wave) HIPCHK(launch_tsqr_tree(r.np, acc_f64, L.m_f64, tr, n, s), "tsqr tree");
        else HIPCHK(launch_tsqr_panel_tree(r.np, acc_f64, L.m_f64, tr, n, s), "tsqr panel tree");
    }
    return FIGARO_OK;
}

// Refinement sweep (mixed form): R <- refined R~ (R~ with normalised row signs in rt).
int run_refine(const figaro_table *A, const figaro_table *B, const Shape &sh, const Layout &L, double *R,
               int64_t ldr, void *ws, hipStream_t s)
{
    Stage st("refine", s);
    HIPCHK(launch_refine(A->data, sh.in_f64, sh.lda, sh.m1, (int)sh.n1, B->data, sh.ldb, sh.m2, (int)sh.n2,
                         groups_of(ws, L), !sh.keyed, at<double>(ws, L.headsB), at<double>(ws, L.rt), (int)sh.N(),
                         at<double>(ws, L.gram), at<double>(ws, L.gy), at<double>(ws, L.partial),
                         L.partial_cap, at<int32_t>(ws, L.failed), R, ldr, s),
           "refinement sweep");
    return FIGARO_OK;
}

int run_r(const figaro_table *A, const figaro_table *B, const Shape &sh, const Layout &L, double *R,
          int64_t ldr, void *ws, hipStream_t s)
{
    const int N = (int)sh.N();
    // A Cartesian product in the two-sided form has one head row: one kernel builds it,
    // merges it into diag(R_TA, R_TB) and normalises the row signs.
    const bool cart_root = sh.two_sided && L.regions[0].skip && L.np_root <= 128;
    int rc = run_compact(A, B, sh, L, ws, s, !cart_root);
    if (rc) return rc;
    const int acc = sh.precision == FIGARO_PLAIN_FP64;
    rc = run_regions(L, acc, ws, s);
    if (rc) return rc;
    if (cart_root) {
        const Region &ra = L.regions[1], &rb = L.regions[2];
        {
            Stage st("tsqr_root", s);
            HIPCHK(launch_merge_cartesian(L.np_root, at<double>(ws, ra.root), ra.np, ra.width,
                                          at<double>(ws, rb.root), rb.np, rb.width, groups_of(ws, L),
                                          at<double>(ws, L.headsA), at<double>(ws, L.headsB),
                                          L.refine ? at<double>(ws, L.rt) : R, L.refine ? N : ldr, s),
                   "cartesian root merge");
        }
        return L.refine ? run_refine(A, B, sh, L, R, ldr, ws, s) : FIGARO_OK;
    }
    // Merge in FP64.
    const Region &r0 = L.regions[0];
    const double *cur = at<double>(ws, r0.root);
    int64_t cur_ld = r0.np;
    RowSrc none{};
    if (sh.two_sided) {
        // The tails' triangles occupy disjoint column ranges, so diag(R_TA, R_TB) is
        // already upper triangular: start from it and absorb the heads (their triangle,
        // or the single head row of a Cartesian product) in one pass.
        const Region &ra = L.regions[1], &rb = L.regions[2];
        double *init = at<double>(ws, L.rtmp[0]);
        double *out = at<double>(ws, L.rtmp[1]);
        Stage st("tsqr_root", s);
        HIPCHK(launch_block_diag(at<double>(ws, ra.root), ra.np, ra.width, at<double>(ws, rb.root), rb.np,
                                 rb.width, init, L.np_root, s),
               "block diagonal");
        Groups g = groups_of(ws, L);
        const RowSrc heads = r0.skip ? RowSrc{at<void>(ws, r0.buf), g.counts + CNT_G, 0, N, 0, N}
                                     : RowSrc{cur, nullptr, N, r0.np, 0, N};
        HIPCHK(launch_tsqr_stream(L.np_root, 1, r0.skip ? L.m_f64 : 1, init, L.np_root, heads, none, 1, N,
                                      r0.skip ? 0 : N, 1, out, (int64_t)N * L.np_root, s),
                   "tsqr merge");
        cur = out;
        cur_ld = L.np_root;
    } else {
        Stage st("tsqr_root", s);
        for (size_t i = 1; i < L.regions.size(); i++) {
            const Region &r = L.regions[i];
            double *out = at<double>(ws, L.rtmp[(i - 1) & 1]);
            RowSrc tri{at<double>(ws, r.root), nullptr, r.width, r.np, r.col_off, r.width};
            HIPCHK(launch_tsqr_stream(L.np_root, 1, 1, cur, cur_ld, tri, none, 1, N, r.width, 1, out,
                                      (int64_t)N * L.np_root, s),
                   "tsqr merge");
            cur = out;
            cur_ld = L.np_root;
        }
    }
    if (!L.refine) {
        Stage st("sign", s);
        HIPCHK(launch_sign_normalise(cur, 1, cur_ld, N, R, ldr, s), "sign normalisation");
        return FIGARO_OK;
    }
    {
        Stage st("sign", s);
        HIPCHK(launch_sign_normalise(cur, 1, cur_ld, N, at<double>(ws, L.rt), N, s), "sign normalisation");
    }
    return run_refine(A, B, sh, L, R, ldr, ws, s);
}

}  // namespace

extern "C" {

const char *figaro_last_error(void) { return g_last_error.c_str(); }

int figaro_r_workspace_size(const figaro_table *A, const figaro_table *B, int32_t precision,
                            size_t *bytes)
{
    Shape sh;
    int rc = make_shape(A, B, precision, &sh);
    if (rc) return rc;
    if (!bytes) return fail(FIGARO_EINVAL, "bytes is NULL");
    *bytes = make_layout(sh).total;
    return FIGARO_OK;
}

int figaro_inspect(const figaro_table *A, const figaro_table *B, int32_t precision, void *ws,
                   size_t ws_bytes, figaro_view *out)
{
    Shape sh;
    int rc = make_shape(A, B, precision, &sh);
    if (rc) return rc;
    Layout L = make_layout(sh);
    rc = check_ws(L, ws, ws_bytes);
    if (rc) return rc;
    if (!out) return fail(FIGARO_EINVAL, "out is NULL");
    Groups g = groups_of(ws, L);
    out->counts = g.counts;
    out->g_key = g.key;
    out->g_offA = g.offA;
    out->g_m1 = g.m1;
    out->g_offB = g.offB;
    out->g_m2 = g.m2;
    out->g_r1 = g.r1;
    out->g_r2 = g.r2;
    out->group_cap = L.gcap;
    out->heads = at<double>(ws, L.headsB);
    out->m1 = at<void>(ws, L.regions[0].buf);
    out->m2 = at<void>(ws, L.regions.back().buf);
    out->heads_a = sh.two_sided ? at<double>(ws, L.headsA) : nullptr;
    out->tails_a = sh.two_sided ? at<void>(ws, L.regions[1].buf) : nullptr;
    out->m_dtype = L.m_f64 ? FIGARO_F64 : FIGARO_F32;
    out->status = at<int32_t>(ws, L.status);
    return FIGARO_OK;
}

int figaro_compact(const figaro_table *A, const figaro_table *B, int32_t precision, void *ws,
                   size_t ws_bytes, void *stream)
{
    Shape sh;
    int rc = make_shape(A, B, precision, &sh);
    if (rc) return rc;
    Layout L = make_layout(sh);
    rc = check_ws(L, ws, ws_bytes);
    if (rc) return rc;
    return run_compact(A, B, sh, L, ws, (hipStream_t)stream);
}

int figaro_r(const figaro_table *A, const figaro_table *B, int32_t precision, double *R,
             int64_t ldr, void *ws, size_t ws_bytes, void *stream)
{
    Shape sh;
    int rc = make_shape(A, B, precision, &sh);
    if (rc) return rc;
    if (!R) return fail(FIGARO_EINVAL, "R is NULL");
    if (ldr < sh.N()) return fail(FIGARO_EINVAL, "ldr < n1 + n2");
    Layout L = make_layout(sh);
    rc = check_ws(L, ws, ws_bytes);
    if (rc) return rc;
    return run_r(A, B, sh, L, R, ldr, ws, (hipStream_t)stream);
}

int figaro_sigma_workspace_size(int64_t n, size_t *bytes)
{
    if (n < 1 || n > FIGARO_MAX_N) return fail(FIGARO_EINVAL, "n out of range");
    if (!bytes) return fail(FIGARO_EINVAL, "bytes is NULL");
    *bytes = kAlign + sizeof(double) * (size_t)std::max(jacobi_scratch_doubles((int)n),
                                                        sigma_bidiag_scratch_doubles((int)n));
    return FIGARO_OK;
}

namespace {

int sigma_common(const double *R, int64_t n, int64_t ldr, double *sigma, void *ws, size_t ws_bytes)
{
    if (n < 1 || n > FIGARO_MAX_N) return fail(FIGARO_EINVAL, "n out of range");
    if (!R || !sigma) return fail(FIGARO_EINVAL, "R or sigma is NULL");
    if (ldr < n) return fail(FIGARO_EINVAL, "ldr < n");
    if (!ws) return fail(FIGARO_EINVAL, "workspace is NULL");
    if (((uintptr_t)ws) % kAlign) return fail(FIGARO_EINVAL, "workspace must be 256-byte aligned");
    size_t need = 0;
    figaro_sigma_workspace_size(n, &need);
    if (ws_bytes < need) return fail(FIGARO_EWORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
    return FIGARO_OK;
}

}  // namespace

namespace {

// `timed`: bracket the launches with stage events (figaro_timing_enable); off for the
// allocation-free entry point, since creating events may allocate.
int sigma_jacobi(const double *R, int64_t n, int64_t ldr, double *sigma, void *ws, hipStream_t stream,
                 bool timed = true)
{
    Stage st(timed ? "jacobi" : nullptr, stream);
    double *scratch = jacobi_scratch_doubles((int)n) ? at<double>(ws, kAlign) : nullptr;
    hipError_t e = launch_jacobi(R, (int)n, ldr, sigma, 60, (int32_t *)ws, scratch, stream);
    if (e != hipSuccess) return hip_fail(e, "jacobi");
    return FIGARO_OK;
}

int sigma_bidiag(const double *R, int64_t n, int64_t ldr, double *sigma, void *ws, hipStream_t stream,
                 bool timed = true)
{
    double *msin = at<double>(ws, kAlign);
    {
        Stage st(timed ? "sigma_bidiag" : nullptr, stream);
        hipError_t e = launch_sigma_bidiag(R, (int)n, ldr, (int32_t *)ws, msin, stream);
        if (e != hipSuccess) return hip_fail(e, "sigma bidiagonalisation");
    }
    Stage st(timed ? "sigma_msect" : nullptr, stream);
    hipError_t e = launch_sigma_msect(msin, (int)n, sigma, stream);
    if (e != hipSuccess) return hip_fail(e, "sigma multisection");
    return FIGARO_OK;
}

}  // namespace

int figaro_sigma(const double *R, int64_t n, int64_t ldr, double *sigma, void *ws, size_t ws_bytes,
                 void *stream)
{
    int rc = sigma_common(R, n, ldr, sigma, ws, ws_bytes);
    if (rc) return rc;
    if (n <= 128) return sigma_bidiag(R, n, ldr, sigma, ws, (hipStream_t)stream);
    return sigma_jacobi(R, n, ldr, sigma, ws, (hipStream_t)stream);
}

int figaro_sigma_jacobi(const double *R, int64_t n, int64_t ldr, double *sigma, void *ws, size_t ws_bytes,
                        void *stream)
{
    int rc = sigma_common(R, n, ldr, sigma, ws, ws_bytes);
    if (rc) return rc;
    return sigma_jacobi(R, n, ldr, sigma, ws, (hipStream_t)stream);
}

int figaro_sigma_bidiag(const double *R, int64_t n, int64_t ldr, double *sigma, void *ws, size_t ws_bytes,
                        void *stream)
{
    int rc = sigma_common(R, n, ldr, sigma, ws, ws_bytes);
    if (rc) return rc;
    if (n > 128) return fail(FIGARO_EINVAL, "the bidiagonal route takes n <= 128");
    return sigma_bidiag(R, n, ldr, sigma, ws, (hipStream_t)stream);
}

// ------------------------------------------------------------ sigma without allocation
//
// The workspace of figaro_sigma for every n <= FIGARO_MAX_N (a 256-byte control block and
// at most 512 x 512 FP64 columns of the block Jacobi) as one device array of the library.
// Every GPU holds its own copy until the process ends; host code reaches it only through
// the address hipGetSymbolAddress returns on that GPU (the array's name is a host-side
// stand-in, not a device address).  Calls on one GPU share it and must not overlap; each
// call clears what its kernels need cleared (the control block is zeroed in-stream by the
// first kernel of either route, the rest is written before it is read).
}  // extern "C"

namespace {

constexpr size_t kNoAllocBytes = kAlign + sizeof(double) * (size_t)FIGARO_MAX_N * FIGARO_MAX_N;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Address of this GPU's copy of `scratch`, looked up once per device with it current.
int scratch_address(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(FIGARO_EINVAL, "device index beyond the supported 64");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p || ((uintptr_t)p) % kAlign) return fail(FIGARO_EHIP, "static scratch address is null or misaligned");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FIGARO_OK;
}

}  // namespace

extern "C" {

int figaro_sigma_noalloc(const double *R, int64_t n, int64_t ldr, double *sigma, void *stream)
{
    if (n < 1 || n > FIGARO_MAX_N)
        return fail(FIGARO_EINVAL, "n out of range [1, 512] (the static scratch holds the workspace of n <= 512)");
    if (!R || !sigma) return fail(FIGARO_EINVAL, "R or sigma is NULL");
    if (ldr < n) return fail(FIGARO_EINVAL, "ldr < n");
    size_t need = 0;
    figaro_sigma_workspace_size(n, &need);
    if (need > kNoAllocBytes) return fail(FIGARO_EINVAL, "workspace of this n exceeds the static scratch");
    void *ws = nullptr;
    int rc = scratch_address(&ws);
    if (rc) return rc;
    if (n <= 128) return sigma_bidiag(R, n, ldr, sigma, ws, (hipStream_t)stream, false);
    return sigma_jacobi(R, n, ldr, sigma, ws, (hipStream_t)stream, false);
}

int figaro_timing_enable(int32_t on)
{
    g_timing.on.store(on != 0);
    return FIGARO_OK;
}

int figaro_timing_read(const char **names, double *ms, int32_t *launches, int32_t cap,
                       int32_t *count)
{
    if (!count) return fail(FIGARO_EINVAL, "count is NULL");
    std::lock_guard<std::mutex> lk(g_timing.mu);
    std::vector<const char *> nm;
    std::vector<double> tot;
    std::vector<int32_t> cnt;
    for (auto &r : g_timing.recs) {
        hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess) return hip_fail(e, "timing sync");
        float t = 0.f;
        e = hipEventElapsedTime(&t, r.a, r.b);
        if (e != hipSuccess) return hip_fail(e, "timing elapsed");
        size_t i = 0;
        while (i < nm.size() && std::strcmp(nm[i], r.name) != 0) i++;
        if (i == nm.size()) {
            nm.push_back(r.name);
            tot.push_back(0.0);
            cnt.push_back(0);
        }
        tot[i] += t;
        cnt[i] += 1;
        g_timing.pool.push_back(r.a);
        g_timing.pool.push_back(r.b);
    }
    g_timing.recs.clear();
    const int n = (int)std::min<size_t>(nm.size(), cap > 0 ? (size_t)cap : 0);
    for (int i = 0; i < n; i++) {
        if (names) names[i] = nm[i];
        if (ms) ms[i] = tot[i];
        if (launches) launches[i] = cnt[i];
    }
    *count = (int32_t)nm.size();
    return FIGARO_OK;
}

int figaro_status(const void *ws, void *stream, int32_t *code)
{
    if (!ws || !code) return fail(FIGARO_EINVAL, "ws or code is NULL");
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "status sync");
    int32_t v = 0;
    e = hipMemcpy(&v, ws, sizeof(v), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "status read");
    *code = v;
    return FIGARO_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ plans

struct figaro_plan {
    std::vector<figaro_instance> inst;
    std::vector<Shape> shapes;
    std::vector<Layout> layouts;
    std::vector<int64_t> r_off, s_off;
    int64_t r_total = 0, s_total = 0;
    size_t ws_bytes = 0;
    size_t lane_bytes = 0;          // workspace slice of one lane
    std::vector<int> lane;          // lane of each instance
    int nlanes = 1;
    hipStream_t cap_stream = nullptr;
    // Batched sigma: per width class, a contiguous run of (r_off, s_off, n, msin offset)
    // entries in the device table `stab` (owned by the plan); the multisection inputs of
    // every instance sit after the lanes' workspace slices.
    int64_t *stab = nullptr;           // uploaded at the first execution (creation is host-only)
    std::vector<int64_t> stab_host;
    std::vector<std::pair<int, std::pair<int, int>>> sclass;  // (class, (first entry, count))
    size_t msin_off = 0;               // byte offset of the multisection inputs in the workspace
    std::vector<hipStream_t> lane_streams;
    std::vector<hipEvent_t> lane_events;  // [0]: fork, [1 + l]: join of lane l
    // One captured graph per (ws, R, sigma) triple.
    std::map<std::tuple<void *, double *, double *>, hipGraphExec_t> graphs;
};

namespace {

// Instances run as nlanes parallel branches: lane l owns workspace slice l and runs its
// instances in order; the branches fork from and join back into s.
int plan_enqueue(figaro_plan *plan, void *ws, double *R, double *sigma, hipStream_t s)
{
    HIPCHK(hipEventRecord(plan->lane_events[0], s), "fork");
    for (int l = 0; l < plan->nlanes; l++)
        HIPCHK(hipStreamWaitEvent(plan->lane_streams[l], plan->lane_events[0], 0), "fork wait");
    for (size_t i = 0; i < plan->inst.size(); i++) {
        const Shape &sh = plan->shapes[i];
        const int64_t N = sh.N();
        const int l = plan->lane[i];
        hipStream_t ls = plan->lane_streams[l];
        void *lws = (char *)ws + (size_t)l * plan->lane_bytes;
        int rc = run_r(&plan->inst[i].A, &plan->inst[i].B, sh, plan->layouts[i], R + plan->r_off[i], N, lws, ls);
        if (rc) return rc;
    }
    for (int l = 0; l < plan->nlanes; l++) {
        HIPCHK(hipEventRecord(plan->lane_events[1 + l], plan->lane_streams[l]), "join");
        HIPCHK(hipStreamWaitEvent(s, plan->lane_events[1 + l], 0), "join wait");
    }
    // sigma of every instance: per width class, one bidiagonalisation workgroup per instance,
    // then one multisection workgroup per singular value
    double *msin = at<double>(ws, plan->msin_off);
    for (const auto &c : plan->sclass)
        HIPCHK(launch_sigma_batch(c.first, R, sigma, plan->stab + 4 * (int64_t)c.second.first, c.second.second, msin,
                                  s),
               "batched sigma");
    return FIGARO_OK;
}

}  // namespace

extern "C" {

int figaro_plan_create(const figaro_instance *inst, int32_t count, int32_t precision,
                       figaro_plan **out)
{
    if (!inst || count < 1 || !out) return fail(FIGARO_EINVAL, "bad plan arguments");
    figaro_plan *p = new figaro_plan();
    size_t wsmax = 0;
    for (int i = 0; i < count; i++) {
        Shape sh;
        int rc = make_shape(&inst[i].A, &inst[i].B, precision, &sh);
        if (rc) {
            delete p;
            return rc;
        }
        if (sh.N() > 128) {
            delete p;
            return fail(FIGARO_EINVAL, "plan instances need n1 + n2 <= 128 in this build");
        }
        Layout L = make_layout(sh);
        p->inst.push_back(inst[i]);
        p->shapes.push_back(sh);
        p->layouts.push_back(L);
        p->r_off.push_back(p->r_total);
        p->s_off.push_back(p->s_total);
        p->r_total += sh.N() * sh.N();
        p->s_total += sh.N();
        wsmax = std::max(wsmax, align_up(L.total));
    }
    // Lanes: largest instances first, each to the lane with the least work so far
    // (work ~ rows x N^2; ties to the lower lane, so the assignment is deterministic).
    p->nlanes = std::min(count, kPlanLanes);
    p->lane.assign(count, 0);
    std::vector<int> order(count);
    for (int i = 0; i < count; i++) order[i] = i;
    auto work = [&](int i) {
        const Shape &sh = p->shapes[i];
        return (double)(sh.m1 + sh.m2) * (double)(sh.N() * sh.N());
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
    std::vector<double> load(p->nlanes, 0.0);
    for (int i : order) {
        const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        p->lane[i] = l;
        load[l] += work(i);
    }
    p->lane_bytes = wsmax;
    p->msin_off = wsmax * p->nlanes;
    // multisection inputs: 2 N + 2 doubles per instance
    p->ws_bytes = p->msin_off + align_up(sizeof(double) * (size_t)(2 * p->s_total + 2 * (int64_t)count));
    // instance table of the batched sigma, grouped by width class
    std::vector<int64_t> tab;
    for (int c = 8; c <= 128; c *= 2) {
        const int first = (int)(tab.size() / 4);
        for (int i = 0; i < count; i++) {
            if (sigma_width_class((int)p->shapes[i].N()) != c) continue;
            tab.push_back(p->r_off[i]);
            tab.push_back(p->s_off[i]);
            tab.push_back(p->shapes[i].N());
            tab.push_back(2 * p->s_off[i] + 2 * (int64_t)i);
        }
        const int n = (int)(tab.size() / 4) - first;
        if (n > 0) p->sclass.push_back({c, {first, n}});
    }
    p->stab_host = std::move(tab);
    *out = p;
    return FIGARO_OK;
}

int figaro_plan_workspace_size(const figaro_plan *plan, size_t *bytes)
{
    if (!plan || !bytes) return fail(FIGARO_EINVAL, "plan or bytes is NULL");
    *bytes = plan->ws_bytes;
    return FIGARO_OK;
}

int figaro_plan_offsets(const figaro_plan *plan, int64_t *r_off, int64_t *s_off, int64_t *r_total,
                        int64_t *s_total)
{
    if (!plan) return fail(FIGARO_EINVAL, "plan is NULL");
    const size_t n = plan->inst.size();
    if (r_off) std::memcpy(r_off, plan->r_off.data(), n * sizeof(int64_t));
    if (s_off) std::memcpy(s_off, plan->s_off.data(), n * sizeof(int64_t));
    if (r_total) *r_total = plan->r_total;
    if (s_total) *s_total = plan->s_total;
    return FIGARO_OK;
}

int figaro_plan_execute(figaro_plan *plan, void *ws, size_t ws_bytes, double *R, double *sigma,
                        void *stream)
{
    if (!plan || !R || !sigma) return fail(FIGARO_EINVAL, "plan, R or sigma is NULL");
    if (!ws) return fail(FIGARO_EINVAL, "workspace is NULL");
    if (((uintptr_t)ws) % kAlign) return fail(FIGARO_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < plan->ws_bytes) return fail(FIGARO_EWORKSPACE, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    auto key = std::make_tuple(ws, R, sigma);
    auto it = plan->graphs.find(key);
    if (!plan->stab) {
        const size_t nb = sizeof(int64_t) * std::max<size_t>(1, plan->stab_host.size());
        HIPCHK(hipMalloc((void **)&plan->stab, nb), "plan instance table");
        HIPCHK(hipMemcpy(plan->stab, plan->stab_host.data(), sizeof(int64_t) * plan->stab_host.size(),
                         hipMemcpyHostToDevice),
               "plan instance table");
    }
    if (it == plan->graphs.end()) {
        if (!plan->cap_stream) {
            HIPCHK(hipStreamCreateWithFlags(&plan->cap_stream, hipStreamNonBlocking), "plan stream");
            plan->lane_streams.assign(plan->nlanes, nullptr);
            for (auto &ls : plan->lane_streams)
                HIPCHK(hipStreamCreateWithFlags(&ls, hipStreamNonBlocking), "plan lane stream");
            plan->lane_events.assign(plan->nlanes + 1, nullptr);
            for (auto &ev : plan->lane_events)
                HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "plan event");
        }
        hipGraph_t graph = nullptr;
        HIPCHK(hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeThreadLocal),
               "begin capture");
        t_capturing = true;
        int rc = plan_enqueue(plan, ws, R, sigma, plan->cap_stream);
        t_capturing = false;
        hipError_t e = hipStreamEndCapture(plan->cap_stream, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "end capture");
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(e, "graph instantiate");
        it = plan->graphs.emplace(key, exec).first;
    }
    Stage st("plan_graph", s);
    HIPCHK(hipGraphLaunch(it->second, s), "graph launch");
    return FIGARO_OK;
}

void figaro_plan_destroy(figaro_plan *plan)
{
    if (!plan) return;
    for (auto &kv : plan->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto ev : plan->lane_events)
        if (ev) (void)hipEventDestroy(ev);
    for (auto ls : plan->lane_streams)
        if (ls) (void)hipStreamDestroy(ls);
    if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);
    if (plan->stab) (void)hipFree(plan->stab);
    delete plan;
}

}  // extern "C"
