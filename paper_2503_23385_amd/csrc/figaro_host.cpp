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
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "common.h"
#include "tune.h"
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
// Wide regions up to this padded width take the streaming panel tree, wider ones the
// blocked QR tree (measured: the panel tree is the faster at 128 on the 2^20-row join,
// the blocked one at 256 and 512 on the 2^18 x 256 join).
constexpr int kPanelTreeMaxNp = 128;
constexpr int kMaxPanelLeaves = 128;
constexpr int kBatchGramBlocks = 64;  // Gram workgroups per job in a batch

struct Shape {
    int64_t m1, n1, lda, m2, n2, ldb;
    int in_f64;
    bool keyed;
    int precision;  // FIGARO_PLAIN_FP64 / FIGARO_MIXED_FP32 / FIGARO_MIXED_FP32_REFINE
    bool two_sided;
    bool givens;    // regions reduced by Givens rotations (FIGARO_GIVENS)
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
    bool wave;                // tuned tree kernel (np <= 128); else the blocked QR tree
    bool wave_tree;           // narrow regions: one wave per leaf (else one workgroup per leaf)
    bool givens;              // narrow regions: leaves absorb rows by Givens rotations
    bool skip;                // rows absorbed directly by the root merge (no tree of its own)
    int leaves, arity;        // most leaves; tree arity
    int64_t nslots, ncnt;     // node triangles and counters reserved (for every tuning candidate)
    int64_t rows_per_leaf;    // leaves follow the device row count: ceil(rows / rows_per_leaf)
    size_t slots, counters, root;
    size_t vbuf;              // wide regions: reflector side buffers, one per leaf
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
    if ((precision & ~(kPrecMask | FIGARO_TWO_SIDED | FIGARO_GIVENS)) != 0 ||
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
    sh->givens = (precision & FIGARO_GIVENS) != 0;
    if (sh->givens) {
        if (prec != FIGARO_PLAIN_FP64) return fail(FIGARO_EINVAL, "the Givens route runs in FP64 only");
        // every region must be narrow: the tails (both forms), region 1 / the head rows
        // (N wide) unless a Cartesian product's single head row goes to the root
        const bool wide_rows = !sh->two_sided || sh->keyed;
        if (A->cols > 64 || B->cols > 64 || (wide_rows && N > 64))
            return fail(FIGARO_EINVAL, "the Givens route takes regions up to 64 columns");
    }
    return FIGARO_OK;
}

int env_int(const char *name, int dflt)
{
    const char *v = std::getenv(name);
    if (!v || !*v) return dflt;
    const int x = std::atoi(v);
    return x > 0 ? x : dflt;
}

constexpr int kMaxWaveLeaves = 1 << 16;

// Tree kernel and leaves of a narrow region under tuning entry t.
void apply_tree(Region &r, const TreeTune &t, int acc_f64)
{
    int64_t leaves;
    if (r.np > 64 && t.kind != TREE_WAVE) {
        // the workgroup kernel of width 128 is the panel tree: rows streamed through LDS
        // into each leaf's triangle, leaves of 4 blocks, binary tree
        r.wave_tree = false;
        r.arity = 2;
        r.rows_per_leaf = (int64_t)4 * tsqr_block_rows(r.np, acc_f64);
        leaves = (r.rows_cap + r.rows_per_leaf - 1) / r.rows_per_leaf;
        r.leaves = (int)std::max<int64_t>(1, std::min<int64_t>(leaves, kMaxPanelLeaves));
        return;
    }
    if (t.kind == TREE_WAVE) {
        r.wave_tree = true;
        r.rows_per_leaf = (int64_t)std::max(1, t.leaf_blocks) * tsqr_wave_block_rows(r.np);
        leaves = (r.rows_cap + r.rows_per_leaf - 1) / r.rows_per_leaf;
        r.leaves = (int)std::max<int64_t>(1, std::min<int64_t>(leaves, kMaxWaveLeaves));
        r.arity = std::max(2, std::min(32, t.arity));
        return;
    }
    r.wave_tree = false;
    const int br = tsqr_block_rows(r.np, acc_f64);
    if (t.leaf_blocks > 0) {
        r.rows_per_leaf = (int64_t)t.leaf_blocks * br;
    } else {
        // default rule (measured): leaves of two blocks, lengthened to keep a region at
        // kLeafTarget leaves (two per compute unit when the two tails share a launch):
        // shorter leaves add workgroups that wait for a compute unit, longer ones add
        // sequential column steps
        const int64_t per_leaf = (r.rows_cap + kLeafTarget - 1) / kLeafTarget;
        r.rows_per_leaf = std::max<int64_t>(2 * br, (per_leaf + br - 1) / br * br);
    }
    leaves = (r.rows_cap + r.rows_per_leaf - 1) / r.rows_per_leaf;
    r.leaves = (int)std::max<int64_t>(1, std::min<int64_t>(leaves, kMaxTreeLeaves));
    r.arity = tsqr_tree_arity(r.np, r.width);
}

// Node slots and counters of a region's tree under its current kernel.
void region_tree_sizes(const Region &r, int64_t *slots, int64_t *counters)
{
    if (r.np > 64 && !r.wave_tree) tsqr_panel_tree_sizes(r.leaves, slots, counters);
    else tsqr_tree_sizes(r.leaves, r.arity, slots, counters);
}

// A region of rows_cap rows reduced by a tree: regions up to padded width 128 take the
// tree kernel and leaf length of the tuning table (at 128 the panel tree or one wave per
// leaf); their node storage is sized for every candidate the autotuner may switch to, so
// that the workspace size does not depend on the tuning.  Wider regions take the blocked
// QR tree.
constexpr int64_t kGivensLeafRows = 256;

Region make_region(const char *name, int64_t rows_cap, int cnt, int width, int col_off, int acc_f64,
                   bool batched = false, bool givens = false)
{
    Region r;
    r.givens = false;
    r.name = name;
    r.rows_cap = std::max<int64_t>(0, rows_cap);
    r.cnt = cnt;
    r.width = width;
    r.col_off = col_off;
    r.np = tsqr_padded_width(width);
    r.wave = r.np <= kPanelTreeMaxNp;  // tuned tree kernel (wave or workgroup / panel tree)
    r.ncounters = 0;
    r.skip = false;
    if (!r.wave) {
        r.wave_tree = false;
        r.arity = 2;
        // blocked QR of each leaf's rows at once: leaves as long as the kernel takes
        // (the regions of a form are stored in FP64 exactly when it accumulates in FP64)
        r.rows_per_leaf = wqr_leaf_rows(acc_f64);
        const int64_t leaves = (r.rows_cap + r.rows_per_leaf - 1) / r.rows_per_leaf;
        r.leaves = (int)std::max<int64_t>(1, leaves);
        tsqr_panel_tree_sizes(r.leaves, &r.nslots, &r.ncnt);
        return r;
    }
    if (givens) {
        // rows absorbed one at a time by one wave per leaf: leaves of a fixed length, binary tree
        r.givens = true;
        r.wave_tree = true;
        r.rows_per_leaf = kGivensLeafRows;
        const int64_t leaves = (r.rows_cap + r.rows_per_leaf - 1) / r.rows_per_leaf;
        r.leaves = (int)std::max<int64_t>(1, std::min<int64_t>(leaves, kMaxWaveLeaves));
        r.arity = 2;
        tsqr_tree_sizes(r.leaves, r.arity, &r.nslots, &r.ncnt);
        return r;
    }
    const TuneKey key{acc_f64, r.np, batched ? 1 : 0, rows_log2(r.rows_cap)};
    std::vector<TreeTune> cands = tune_candidates(key);
    cands.push_back(tune_default(key));
    r.nslots = r.ncnt = 0;
    for (const TreeTune &t : cands) {
        Region c = r;
        apply_tree(c, t, acc_f64);
        int64_t ns = 0, nc = 0;
        region_tree_sizes(c, &ns, &nc);
        r.nslots = std::max(r.nslots, ns);
        r.ncnt = std::max(r.ncnt, nc);
    }
    apply_tree(r, tune_get(key), acc_f64);
    int64_t ns = 0, nc = 0;
    region_tree_sizes(r, &ns, &nc);
    r.nslots = std::max(r.nslots, ns);
    r.ncnt = std::max(r.ncnt, nc);
    return r;
}

Layout make_layout(const Shape &s, bool batched = false)
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
        Region a = make_region("tsqr_m1", s.m1, CNT_R1, N, 0, L.m_f64, batched, s.givens);
        Region b = make_region("tsqr_m2", s.m2 - 1, CNT_R2, (int)s.n2, (int)s.n1, L.m_f64, batched, s.givens);
        a.buf = take(esz * std::max<int64_t>(1, a.rows_cap) * N);
        b.buf = take(esz * std::max<int64_t>(1, b.rows_cap) * s.n2);
        L.regions = {a, b};
    } else {
        Region h = make_region("tsqr_heads", L.gcap, CNT_G, N, 0, L.m_f64, batched, s.givens);
        // Cartesian product: a single head row, absorbed by the root merge itself.
        h.skip = !s.keyed;
        Region ta = make_region("tsqr_ta", s.m1 - 1, CNT_TA, (int)s.n1, 0, L.m_f64, batched, s.givens);
        Region tb = make_region("tsqr_tb", s.m2 - 1, CNT_R2, (int)s.n2, (int)s.n1, L.m_f64, batched, s.givens);
        h.buf = take(esz * h.rows_cap * N);
        ta.buf = take(esz * std::max<int64_t>(1, ta.rows_cap) * s.n1);
        tb.buf = take(esz * std::max<int64_t>(1, tb.rows_cap) * s.n2);
        L.regions = {h, ta, tb};
    }
    int64_t ctot = 0;
    for (Region &r : L.regions) {
        const size_t tsz = sizeof(double) * (size_t)r.width * r.np;
        const int64_t ns = r.nslots, nc = r.ncnt;
        r.slots = take(tsz * ns);
        r.ncounters = nc;
        r.counters = (size_t)ctot;  // index into the shared counter block
        ctot += nc;
        r.root = take(tsz);
        r.vbuf = (r.wave || r.np <= kPanelTreeMaxNp) ? 0 : take((size_t)wqr_vbuf_bytes() * (size_t)r.leaves);
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

// Grouping stage: the group table, counts and status, and zeroed tree counters.
int run_grouping(const figaro_table *A, const figaro_table *B, const Shape &sh, const Layout &L, void *ws,
                 hipStream_t s)
{
    Groups g = groups_of(ws, L);
    int32_t *status = at<int32_t>(ws, L.status);
    Stage st("group", s);
    if (sh.keyed) {
        HIPCHK(launch_group_init(status, g.counts, nullptr, at<int32_t>(ws, L.counters_base), L.counters_total, s),
               "init");
        HIPCHK(launch_group_keys(A->keys, sh.m1, B->keys, sh.m2, g, at<int32_t>(ws, L.blkA), at<int32_t>(ws, L.blkB),
                                 at<int32_t>(ws, L.runA), at<int32_t>(ws, L.runB), at<int32_t>(ws, L.matchA),
                                 at<int32_t>(ws, L.blkM), at<int64_t>(ws, L.blkS), status, s),
               "grouping");
    } else {
        HIPCHK(launch_group_cartesian(status, at<int32_t>(ws, L.counters_base), L.counters_total, g, sh.m1, sh.m2,
                                      s),
               "grouping");
    }
    return FIGARO_OK;
}

// The head/tail scan jobs of one problem: B's (both forms), then A's (two-sided form).
int scan_jobs(const figaro_table *A, const figaro_table *B, const Shape &sh, const Layout &L, void *ws,
              ScanJob *jobs)
{
    Groups g = groups_of(ws, L);
    const Region &rb = L.regions.back();  // region of B's tails in both forms
    ScanSide sideB{g.offB, g.m2, g.m1, g.r2, 0};
    jobs[0] = scan_job(B->data, sh.ldb, sh.m2, sh.n2, sideB, at<void>(ws, rb.buf), at<double>(ws, L.headsB),
                       at<int32_t>(ws, L.tileF[1]), at<double>(ws, L.tileS[1]), at<double>(ws, L.carry[1]), L.spB);
    int n = 1;
    if (sh.two_sided) {
        ScanSide sideA{g.offA, g.m1, g.m2, g.r1, 1};
        jobs[1] = scan_job(A->data, sh.lda, sh.m1, sh.n1, sideA, at<void>(ws, L.regions[1].buf),
                           at<double>(ws, L.headsA), at<int32_t>(ws, L.tileF[0]), at<double>(ws, L.tileS[0]),
                           at<double>(ws, L.carry[0]), L.spA);
        n = 2;
    }
    for (int i = 0; i < n; i++) {
        jobs[i].g = g;
        jobs[i].cartesian = !sh.keyed;
    }
    return n;
}

// Region-1 assembly (Claim 1 form) or the head rows (two-sided form), after the scans.
int run_assembly(const figaro_table *A, const Shape &sh, const Layout &L, void *ws, hipStream_t s)
{
    Groups g = groups_of(ws, L);
    Stage st("assemble", s);
    if (!sh.two_sided) {
        HIPCHK(launch_assemble_a(A->data, sh.in_f64, sh.lda, sh.m1, sh.n1, sh.n2, g, !sh.keyed,
                                 at<double>(ws, L.headsB), at<void>(ws, L.regions[0].buf), L.m_f64, s),
               "region-1 assembly");
    } else {
        HIPCHK(launch_head_rows(g, L.gcap, at<double>(ws, L.headsA), at<double>(ws, L.headsB), sh.n1, sh.n2,
                                at<void>(ws, L.regions[0].buf), L.m_f64, s),
               "head rows");
    }
    return FIGARO_OK;
}

// Grouping, head/tail scans and assembly: fills the regions' row buffers (the head rows
// of the two-sided form only when head_rows is set).
int run_compact(const figaro_table *A, const figaro_table *B, const Shape &sh, const Layout &L,
                void *ws, hipStream_t s, bool head_rows = true)
{
    int rc = run_grouping(A, B, sh, L, ws, s);
    if (rc) return rc;
    ScanJob jobs[2];
    const int nj = scan_jobs(A, B, sh, L, ws, jobs);
    const ScanJob none{};
    Groups g = groups_of(ws, L);
    static const char *const pass_name[3] = {"scan_reduce", "scan_carry", "scan_write"};
    for (int pass = 0; pass < 3; pass++) {
        // both tables in one launch per pass when their tiles have the same column layout
        Stage st(pass_name[pass], s);
        if (nj == 2 && L.spA.cpt == L.spB.cpt) {
            HIPCHK(launch_seg_scan(jobs[0], jobs[1], L.spB.cpt, sh.in_f64, L.m_f64, g, !sh.keyed, s, pass),
                   "head/tail scans");
        } else {
            HIPCHK(launch_seg_scan(jobs[0], none, L.spB.cpt, sh.in_f64, L.m_f64, g, !sh.keyed, s, pass),
                   "head/tail scan of B");
            if (nj == 2)
                HIPCHK(launch_seg_scan(jobs[1], none, L.spA.cpt, sh.in_f64, L.m_f64, g, !sh.keyed, s, pass),
                       "head/tail scan of A");
        }
    }
    if (!sh.two_sided || head_rows) return run_assembly(A, sh, L, ws, s);
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
    t.vbuf = (r.wave || r.np <= kPanelTreeMaxNp) ? nullptr : at<void>(ws, r.vbuf);
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
            if (!done[j] && !L.regions[j].skip && L.regions[j].np == r.np &&
                L.regions[j].wave_tree == r.wave_tree && L.regions[j].givens == r.givens) {
                tr[n++] = tree_region(L.regions[j], L, ws);
                done[j] = true;
                name = "tsqr_tails";
            }
        }
        Stage st(name, s);
        if (r.givens) HIPCHK(launch_givens_tree(r.np, L.m_f64, tr, n, s), "givens tree");
        else if (r.wave) HIPCHK(launch_tsqr_tree(r.np, acc_f64, L.m_f64, tr, n, s, r.wave_tree), "tsqr tree");
        else HIPCHK(launch_wqr_tree(r.np, L.m_f64, tr, n, s), "wide tsqr tree");
    }
    return FIGARO_OK;
}

// Refinement sweep (mixed form): R <- refined R~ (R~ with normalised row signs in rt).
int run_refine(const figaro_table *A, const figaro_table *B, const Shape &sh, const Layout &L, double *R,
               int64_t ldr, void *ws, hipStream_t s)
{
    for (int part = 0; part < 2; part++) {
        Stage st(part == 0 ? "refine_gram" : "refine_solve", s);
        HIPCHK(launch_refine(A->data, sh.in_f64, sh.lda, sh.m1, (int)sh.n1, B->data, sh.ldb, sh.m2, (int)sh.n2,
                             groups_of(ws, L), !sh.keyed, sh.two_sided ? at<double>(ws, L.headsA) : nullptr,
                             at<double>(ws, L.headsB), L.gcap, at<double>(ws, L.rt), (int)sh.N(),
                             at<double>(ws, L.gram), at<double>(ws, L.gy), at<double>(ws, L.partial),
                             L.partial_cap, at<int32_t>(ws, L.failed), R, ldr, s, part),
               "refinement sweep");
    }
    return FIGARO_OK;
}

// A Cartesian product in the two-sided form has one head row: one kernel builds it,
// merges it into diag(R_TA, R_TB) and normalises the row signs.
bool cartesian_root(const Shape &sh, const Layout &L)
{
    return sh.two_sided && L.regions[0].skip && L.np_root <= 128;
}

// Everything after the regions' trees: the merge of their triangles, the row signs and
// the refinement sweep.
// refine = false: the refined forms leave R~ (signs normalised) in the workspace for a
// batched refinement sweep.
int run_root(const figaro_table *A, const figaro_table *B, const Shape &sh, const Layout &L, double *R,
             int64_t ldr, void *ws, hipStream_t s, bool refine = true)
{
    const int N = (int)sh.N();
    if (cartesian_root(sh, L)) {
        const Region &ra = L.regions[1], &rb = L.regions[2];
        {
            Stage st("tsqr_root", s);
            HIPCHK(launch_merge_cartesian(L.np_root, at<double>(ws, ra.root), ra.np, ra.width,
                                          at<double>(ws, rb.root), rb.np, rb.width, groups_of(ws, L),
                                          at<double>(ws, L.headsA), at<double>(ws, L.headsB),
                                          L.refine ? at<double>(ws, L.rt) : R, L.refine ? N : ldr, s),
                   "cartesian root merge");
        }
        return L.refine && refine ? run_refine(A, B, sh, L, R, ldr, ws, s) : FIGARO_OK;
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
        if (!r0.skip && L.np_root > kPanelTreeMaxNp) {
            // wide: the heads' triangle merged into diag(R_TA, R_TB) in place
            HIPCHK(launch_wqr_merge(init, L.np_root, at<double>(ws, r0.root), r0.np, N, at<double>(ws, r0.vbuf), s),
                   "wide root merge");
            cur = init;
        } else {
            Groups g = groups_of(ws, L);
            const RowSrc heads = r0.skip ? RowSrc{at<void>(ws, r0.buf), g.counts + CNT_G, 0, N, 0, N}
                                         : RowSrc{cur, nullptr, N, r0.np, 0, N};
            HIPCHK(launch_tsqr_stream(L.np_root, 1, r0.skip ? L.m_f64 : 1, init, L.np_root, heads, none, 1, N,
                                      r0.skip ? 0 : N, 1, out, (int64_t)N * L.np_root, s),
                   "tsqr merge");
            cur = out;
        }
        cur_ld = L.np_root;
    } else {
        Stage st("tsqr_root", s);
        for (size_t i = 1; i < L.regions.size(); i++) {
            const Region &r = L.regions[i];
            if (L.np_root > kPanelTreeMaxNp) {
                // wide: region i's triangle, placed at its columns, merged into region 0's root
                double *pad = at<double>(ws, L.rtmp[0]);
                HIPCHK(launch_wqr_pad(at<double>(ws, r.root), r.np, r.width, r.col_off, pad, L.np_root, N, s),
                       "pad triangle");
                HIPCHK(launch_wqr_merge(at<double>(ws, r0.root), r0.np, pad, L.np_root, N, at<double>(ws, r0.vbuf), s),
                       "wide root merge");
                continue;
            }
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
    return refine ? run_refine(A, B, sh, L, R, ldr, ws, s) : FIGARO_OK;
}

int run_r(const figaro_table *A, const figaro_table *B, const Shape &sh, const Layout &L, double *R,
          int64_t ldr, void *ws, hipStream_t s)
{
    int rc = run_compact(A, B, sh, L, ws, s, !cartesian_root(sh, L));
    if (rc) return rc;
    rc = run_regions(L, sh.precision == FIGARO_PLAIN_FP64, ws, s);
    if (rc) return rc;
    return run_root(A, B, sh, L, R, ldr, ws, s);
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

int figaro_sigma_dqds(const double *R, int64_t n, int64_t ldr, double *sigma, void *ws, size_t ws_bytes,
                      void *stream)
{
    int rc = sigma_common(R, n, ldr, sigma, ws, ws_bytes);
    if (rc) return rc;
    if (n > 128) return fail(FIGARO_EINVAL, "the dqds route takes n <= 128");
    hipStream_t st = (hipStream_t)stream;
    double *msin = at<double>(ws, kAlign);
    {
        Stage sg("sigma_bidiag", st);
        hipError_t e = launch_sigma_bidiag(R, (int)n, ldr, (int32_t *)ws, msin, st);
        if (e != hipSuccess) return hip_fail(e, "sigma bidiagonalisation");
    }
    Stage sg("sigma_dqds", st);
    hipError_t e = launch_sigma_dqds(msin, (int)n, sigma, st);
    if (e != hipSuccess) return hip_fail(e, "dqds");
    return FIGARO_OK;
}

int figaro_sigma_bidiag(const double *R, int64_t n, int64_t ldr, double *sigma, void *ws, size_t ws_bytes,
                        void *stream)
{
    int rc = sigma_common(R, n, ldr, sigma, ws, ws_bytes);
    if (rc) return rc;
    if (n > 128) return fail(FIGARO_EINVAL, "the bidiagonal route takes n <= 128");
    return sigma_bidiag(R, n, ldr, sigma, ws, (hipStream_t)stream);
}

int figaro_svd_workspace_size(int64_t n, size_t *bytes)
{
    if (n < 1 || n > 128) return fail(FIGARO_EINVAL, "n out of range [1, 128] for the singular vectors");
    if (!bytes) return fail(FIGARO_EINVAL, "bytes is NULL");
    *bytes = kAlign + sizeof(double) * (size_t)svd_v_scratch_doubles((int)n);
    return FIGARO_OK;
}

int figaro_svd(const double *R, int64_t n, int64_t ldr, double *sigma, double *V, int64_t ldv, void *ws,
               size_t ws_bytes, void *stream)
{
    if (n < 1 || n > 128) return fail(FIGARO_EINVAL, "n out of range [1, 128] for the singular vectors");
    if (!R || !sigma || !V) return fail(FIGARO_EINVAL, "R, sigma or V is NULL");
    if (ldr < n || ldv < n) return fail(FIGARO_EINVAL, "ldr or ldv < n");
    if (!ws) return fail(FIGARO_EINVAL, "workspace is NULL");
    if (((uintptr_t)ws) % kAlign) return fail(FIGARO_EINVAL, "workspace must be 256-byte aligned");
    size_t need = 0;
    figaro_svd_workspace_size(n, &need);
    if (ws_bytes < need) return fail(FIGARO_EWORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
    Stage st("svd_v", (hipStream_t)stream);
    hipError_t e = launch_svd_v(R, (int)n, ldr, sigma, V, ldv, 60, (int32_t *)ws, at<double>(ws, kAlign),
                                (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "singular vectors");
    return FIGARO_OK;
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

int figaro_sort_workspace_size(int64_t rows, size_t *bytes)
{
    if (rows < 0 || rows > INT32_MAX - 1) return fail(FIGARO_EINVAL, "rows out of range");
    if (!bytes) return fail(FIGARO_EINVAL, "bytes is NULL");
    *bytes = (size_t)sort_workspace_bytes(rows);
    return FIGARO_OK;
}

int figaro_sort_table(const figaro_table *in, void *out, int64_t ld_out, int32_t *keys_out, void *ws,
                      size_t ws_bytes, void *stream)
{
    int rc = check_table(in, "in");
    if (rc) return rc;
    if (!in->keys && in->rows > 0) return fail(FIGARO_EINVAL, "the table has no keys to sort by");
    if (in->rows > 0 && (!out || !keys_out)) return fail(FIGARO_EINVAL, "out or keys_out is NULL");
    if (ld_out < in->cols) return fail(FIGARO_EINVAL, "ld_out < cols");
    if (out == in->data) return fail(FIGARO_EINVAL, "out must not alias the input rows");
    if (!ws) return fail(FIGARO_EINVAL, "workspace is NULL");
    if (((uintptr_t)ws) % kAlign) return fail(FIGARO_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < (size_t)sort_workspace_bytes(in->rows))
        return fail(FIGARO_EWORKSPACE, "workspace too small: need " + std::to_string(sort_workspace_bytes(in->rows)));
    Stage st("sort", (hipStream_t)stream);
    HIPCHK(launch_sort_table(in->data, in->dtype == FIGARO_F64 ? 8 : 4, in->ld, in->rows, in->cols, in->keys, out,
                             ld_out, keys_out, ws, (hipStream_t)stream),
           "sort");
    return FIGARO_OK;
}

int figaro_memory_report(const figaro_table *A, const figaro_table *B, int32_t precision, const void *ws,
                         size_t ws_bytes, void *stream, figaro_memory *out)
{
    Shape sh;
    int rc = make_shape(A, B, precision, &sh);
    if (rc) return rc;
    if (!out) return fail(FIGARO_EINVAL, "out is NULL");
    Layout L = make_layout(sh);
    rc = check_ws(L, const_cast<void *>(ws), ws_bytes);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize((hipStream_t)stream), "memory report sync");
    int64_t counts[CNT_SLOTS];
    HIPCHK(hipMemcpy(counts, (const char *)ws + L.counts, sizeof counts, hipMemcpyDeviceToHost), "memory report read");
    const int64_t N = sh.N();
    const double esz_in = sh.in_f64 ? 8.0 : 4.0, esz_m = L.m_f64 ? 8.0 : 4.0;
    out->groups = counts[CNT_G];
    out->join_rows = counts[CNT_JOIN];
    double compact = 0.0;
    int64_t crows = 0;
    if (!sh.two_sided) {
        crows = counts[CNT_R1] + counts[CNT_R2];
        compact = esz_m * ((double)counts[CNT_R1] * N + (double)counts[CNT_R2] * sh.n2);
    } else {
        crows = counts[CNT_G] + counts[CNT_TA] + counts[CNT_R2];
        compact = esz_m * ((double)counts[CNT_G] * N + (double)counts[CNT_TA] * sh.n1 + (double)counts[CNT_R2] * sh.n2);
    }
    out->compact_rows = crows;
    out->input_bytes = esz_in * ((double)sh.m1 * sh.n1 + (double)sh.m2 * sh.n2) +
                       (sh.keyed ? 4.0 * (double)(sh.m1 + sh.m2) : 0.0);
    out->compact_bytes = compact;
    out->workspace_bytes = (double)L.total;
    out->join_bytes = esz_in * (double)counts[CNT_JOIN] * (double)N;
    return FIGARO_OK;
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
//
// A plan runs its instances stage by stage: each stage is one launch (or one short
// sequence) over every instance at once, driven by device tables of per-instance
// descriptors, so that the batch fills the GPU rather than any one instance:
//   1. grouping: one launch for all Cartesian instances (their one-group tables and
//      zeroed tree counters); a keyed instance runs its own grouping launches;
//   2. head/tail scans: one three-launch sequence (tile reduce, carry scan, tile write)
//      over the tiles of every instance's tables, per (columns per thread, input type);
//   3. region assembly where the form needs it (per instance);
//   4. TSQR: one tree launch per padded width <= 64 over the leaves of every region of
//      every instance (each region with its own node counters and root); wider regions
//      run their own panel-tree launches;
//   5. roots: one launch per padded width over the Cartesian two-sided instances; the
//      others (and the refinement sweep) per instance;
//   6. sigma: two launches per width class over all instances (bidiagonal route).
// Each instance owns one slice of the workspace.

struct figaro_plan {
    std::vector<figaro_instance> inst;
    std::vector<Shape> shapes;
    std::vector<Layout> layouts;
    std::vector<size_t> ws_off;        // each instance's workspace slice
    std::vector<int64_t> r_off, s_off;
    int64_t r_total = 0, s_total = 0;
    size_t ws_bytes = 0;
    size_t msin_off = 0;               // multisection inputs of every instance (2 N_i + 2 doubles each)
    hipStream_t cap_stream = nullptr;
    // Side streams (default priority) and events of the sigma stage, whose width classes
    // run side by side: each class fills only part of the GPU (a workgroup per instance).
    static constexpr int kSide = 4;
    int chains = 0;  // run the two chains side by side (from the tuning table; set by the autotuner)
    hipStream_t side[kSide] = {};
    hipEvent_t ev_fork = nullptr;
    hipEvent_t ev_join[kSide] = {};
    // Per (ws, R, sigma): the device launch tables (built and uploaded when that triple
    // is first executed, owned by the plan) and the captured graph.
    struct Exec {
        unsigned char *tables = nullptr;
        hipGraphExec_t graph = nullptr;
    };
    std::map<std::tuple<void *, double *, double *>, Exec> execs;
};

namespace {

// Host image of a plan's device tables, each array 256-byte aligned; offsets are
// relative to the start of the device allocation.
struct TableImage {
    std::vector<unsigned char> bytes;
    template <typename T>
    size_t add(const std::vector<T> &v)
    {
        const size_t off = align_up(bytes.size());
        bytes.resize(off + std::max<size_t>(1, v.size() * sizeof(T)));
        if (!v.empty()) std::memcpy(bytes.data() + off, v.data(), v.size() * sizeof(T));
        return off;
    }
};

// Stage names of the batched launches, by padded width (4 .. 512).
const char *class_name(const char *const (&names)[8], int np)
{
    int i = 0;
    while (i < 7 && (4 << i) < np) i++;
    return names[i];
}
const char *const kTreeNames[8] = {"tsqr_np4", "tsqr_np8", "tsqr_np16", "tsqr_np32",
                                   "tsqr_np64", "tsqr_np128", "tsqr_np256", "tsqr_np512"};
const char *const kRootNames[8] = {"root_np4", "root_np8", "root_np16", "root_np32",
                                   "root_np64", "root_np128", "root_np256", "root_np512"};
const char *const kSigmaNames[8] = {"sigma_np4", "sigma_np8", "sigma_np16", "sigma_np32",
                                    "sigma_np64", "sigma_np128", "sigma_np256", "sigma_np512"};

// One step of a batch: enqueues its launches given the device address of the tables.
using Step = std::function<int(const unsigned char *tables, hipStream_t s)>;

struct Program {
    TableImage img;
    std::vector<Step> steps;
    std::vector<int> lanes;  // per step: 0 the launch stream, k > 0 the plan's side stream k - 1
    int lane = 0;            // lane of the steps pushed from now on
    const figaro_plan *plan = nullptr;
    void set_lane(int k)
    {
        lanes.resize(steps.size(), lane);
        lane = k;
    }
};

// The steps and tables of one execution of the plan with these buffers.
// fuse_trees: the wave-tree classes of every width share one launch (the autotuner times
// each class in a launch of its own).
Program build_program(const figaro_plan *plan, void *ws, double *R, double *sigma, bool fuse_trees = true)
{
    Program P;
    P.plan = plan;
    const size_t count = plan->inst.size();
    const int prec = plan->shapes[0].precision;
    const int acc = prec == FIGARO_PLAIN_FP64;
    const int m_f64 = acc;
    auto slice = [&](size_t i) { return (void *)((char *)ws + plan->ws_off[i]); };

    // 1. grouping
    std::vector<CartInit> inits;
    for (size_t i = 0; i < count; i++) {
        const Shape &sh = plan->shapes[i];
        const Layout &L = plan->layouts[i];
        void *lws = slice(i);
        if (sh.keyed) {
            const figaro_instance *in = &plan->inst[i];
            P.steps.push_back([in, sh, &L, lws](const unsigned char *, hipStream_t s) {
                return run_grouping(&in->A, &in->B, sh, L, lws, s);
            });
        } else {
            inits.push_back(CartInit{at<int32_t>(lws, L.status), at<int32_t>(lws, L.counters_base),
                                     L.counters_total, groups_of(lws, L), sh.m1, sh.m2});
        }
    }
    if (!inits.empty()) {
        const size_t off = P.img.add(inits);
        const int n = (int)inits.size();
        P.steps.push_back([off, n](const unsigned char *t, hipStream_t s) {
            Stage st("group", s);
            HIPCHK(launch_group_cartesian_batch((const CartInit *)(t + off), n, s), "batched grouping");
            return FIGARO_OK;
        });
    }

    // 2. head/tail scans, per (cpt, input type)
    std::map<std::pair<int, int>, std::vector<ScanJob>> scan_cls;
    for (size_t i = 0; i < count; i++) {
        const Shape &sh = plan->shapes[i];
        const Layout &L = plan->layouts[i];
        ScanJob jobs[2];
        const int nj = scan_jobs(&plan->inst[i].A, &plan->inst[i].B, sh, L, slice(i), jobs);
        const ScanPlan *sp[2] = {&L.spB, &L.spA};
        for (int j = 0; j < nj; j++)
            if (jobs[j].ntiles > 0) scan_cls[{sp[j]->cpt, sh.in_f64}].push_back(jobs[j]);
    }
    for (auto &kv : scan_cls) {
        const std::vector<ScanJob> &jobs = kv.second;
        std::vector<int2> tiles, cols;
        for (int j = 0; j < (int)jobs.size(); j++) {
            for (int64_t t = 0; t < jobs[j].ntiles; t++) tiles.push_back(make_int2(j, (int)t));
            for (int c = 0; c < jobs[j].n; c += 64) cols.push_back(make_int2(j, c));  // 64 columns per carry block
        }
        const size_t jo = P.img.add(jobs), to = P.img.add(tiles), co = P.img.add(cols);
        const int64_t nt = (int64_t)tiles.size(), nc = (int64_t)cols.size();
        const int cpt = kv.first.first, in_f64 = kv.first.second;
        static const char *const pass_name[3] = {"scan_reduce", "scan_carry", "scan_write"};
        for (int pass = 0; pass < 3; pass++) {
            P.steps.push_back([=](const unsigned char *t, hipStream_t s) {
                Stage st(pass_name[pass], s);
                HIPCHK(launch_seg_scan_batch(pass, (const ScanJob *)(t + jo), (const int2 *)(t + to), nt,
                                             (const int2 *)(t + co), nc, cpt, in_f64, m_f64, s),
                       "batched head/tail scans");
                return FIGARO_OK;
            });
        }
    }

    // 3. assembly (Claim 1 region 1; head rows of keyed two-sided instances)
    for (size_t i = 0; i < count; i++) {
        const Shape &sh = plan->shapes[i];
        const Layout &L = plan->layouts[i];
        if (cartesian_root(sh, L)) continue;
        const figaro_instance *in = &plan->inst[i];
        void *lws = slice(i);
        P.steps.push_back([in, sh, &L, lws](const unsigned char *, hipStream_t s) {
            return run_assembly(&in->A, sh, L, lws, s);
        });
    }

    // 4-6. trees, roots, (refinement,) sigma.  Without refinement the instances of sigma
    // width class 128 and the others form two chains that run side by side on the plan's
    // side streams (forked after the assembly, joined at the end): one chain's
    // bidiagonalisations then overlap the other's trees.
    auto emit_trees = [&](const std::vector<size_t> &idx, const char *narrow_name) {
        // 4. trees: narrow regions batched by padded width, wide ones per region
        std::map<std::pair<int, int>, std::vector<TreeRegion>> tree_cls;
        for (size_t i : idx) {
            const Layout &L = plan->layouts[i];
            void *lws = slice(i);
            for (const Region &r : L.regions) {
                if (r.skip || r.rows_cap == 0) continue;
                if (r.wave && r.np <= 64) {
                    tree_cls[{r.np, r.wave_tree ? 1 : 0}].push_back(tree_region(r, L, lws));
                } else {
                    // width 128 (wave or panel tree, by the tuning) and wider: a launch per region
                    const TreeRegion tr = tree_region(r, L, lws);
                    const int np = r.np, wave_tree = r.wave_tree ? 1 : 0;
                    const char *name = r.wave ? class_name(kTreeNames, np) : r.name;
                    P.steps.push_back([tr, np, wave_tree, name, acc, m_f64](const unsigned char *, hipStream_t s) {
                        Stage st(name, s);
                        if (np <= kPanelTreeMaxNp) HIPCHK(launch_tsqr_tree(np, acc, m_f64, &tr, 1, s, wave_tree), "tsqr tree");
                        else HIPCHK(launch_wqr_tree(np, m_f64, &tr, 1, s), "wide tsqr tree");
                        return FIGARO_OK;
                    });
                }
            }
        }
        if (fuse_trees) {
            // every wave-tree class in one launch, the widest leaves first
            std::vector<TreeRegion> regs;
            std::vector<int4> map;
            for (auto it = tree_cls.rbegin(); it != tree_cls.rend(); ++it) {
                if (!it->first.second) continue;
                const int np = it->first.first;
                for (const TreeRegion &tr : it->second) {
                    const int j = (int)regs.size();
                    regs.push_back(tr);
                    for (int l = 0; l < tr.nleaves; l++) map.push_back(make_int4(j, l, np, 0));
                }
            }
            for (auto it = tree_cls.begin(); it != tree_cls.end();) {
                if (it->first.second) it = tree_cls.erase(it);
                else ++it;
            }
            if (!map.empty()) {
                const size_t ro = P.img.add(regs), mo = P.img.add(map);
                const int64_t nb = (int64_t)map.size();
                P.steps.push_back([=](const unsigned char *t, hipStream_t s) {
                    Stage st(narrow_name, s);
                    HIPCHK(launch_tsqr_wtree_multi(acc, m_f64, (const TreeRegion *)(t + ro), (const int4 *)(t + mo), nb,
                                                   s),
                           "batched tsqr trees");
                    return FIGARO_OK;
                });
            }
        }
        for (auto &kv : tree_cls) {
            const std::vector<TreeRegion> &regs = kv.second;
            std::vector<int2> map;
            for (int j = 0; j < (int)regs.size(); j++)
                for (int l = 0; l < regs[j].nleaves; l++) map.push_back(make_int2(j, l));
            const size_t ro = P.img.add(regs), mo = P.img.add(map);
            const int64_t nb = (int64_t)map.size();
            const int np = kv.first.first, wave_tree = kv.first.second;
            const char *name = class_name(kTreeNames, np);
            P.steps.push_back([=](const unsigned char *t, hipStream_t s) {
                Stage st(name, s);
                HIPCHK(launch_tsqr_tree_batch(wave_tree, np, acc, m_f64, (const TreeRegion *)(t + ro),
                                              (const int2 *)(t + mo), nb, s),
                       "batched tsqr tree");
                return FIGARO_OK;
            });
        }

    };
    auto emit_roots = [&](const std::vector<size_t> &idx) {
        // 5. roots: Cartesian two-sided instances batched by padded width, the rest per instance
        std::map<int, std::vector<CartRoot>> root_cls;
        for (size_t i : idx) {
            const Shape &sh = plan->shapes[i];
            const Layout &L = plan->layouts[i];
            void *lws = slice(i);
            const int N = (int)sh.N();
            double *Ri = R + plan->r_off[i];
            if (cartesian_root(sh, L)) {
                const Region &ra = L.regions[1], &rb = L.regions[2];
                root_cls[L.np_root].push_back(CartRoot{at<double>(lws, ra.root), ra.np, ra.width, at<double>(lws, rb.root),
                                                       rb.np, rb.width, groups_of(lws, L), at<double>(lws, L.headsA),
                                                       at<double>(lws, L.headsB), L.refine ? at<double>(lws, L.rt) : Ri,
                                                       L.refine ? N : (int64_t)N});
            } else {
                const figaro_instance *in = &plan->inst[i];
                P.steps.push_back([in, sh, &L, Ri, N, lws](const unsigned char *, hipStream_t s) {
                    return run_root(&in->A, &in->B, sh, L, Ri, N, lws, s, false);
                });
            }
        }
        for (auto &kv : root_cls) {
            const size_t off = P.img.add(kv.second);
            const int n = (int)kv.second.size(), np = kv.first;
            const char *name = class_name(kRootNames, np);
            P.steps.push_back([=](const unsigned char *t, hipStream_t s) {
                Stage st(name, s);
                HIPCHK(launch_merge_cartesian_batch(np, (const CartRoot *)(t + off), n, s), "batched cartesian roots");
                return FIGARO_OK;
            });
        }
    };
    auto emit_sigma = [&](const std::vector<size_t> &idx, bool fork_sigma) {
        // 6. sigma: per width class, one bidiagonalisation workgroup per instance, then one
        // multisection workgroup per singular value; the classes on the plan's side streams
        // (forked from and joined back into the launch stream), widest first
        struct SigmaClass {
            int c, n, dqds;
            size_t off;
            const char *name;
        };
        std::vector<SigmaClass> scls;
        for (int c = 128; c >= 8; c /= 2) {
            std::vector<int64_t> tab;
            for (size_t i : idx) {
                if (sigma_width_class((int)plan->shapes[i].N()) != c) continue;
                tab.push_back(plan->r_off[i]);
                tab.push_back(plan->s_off[i]);
                tab.push_back(plan->shapes[i].N());
                tab.push_back(2 * plan->s_off[i] + 2 * (int64_t)i);
            }
            if (tab.empty()) continue;
            scls.push_back(SigmaClass{c, (int)(tab.size() / 4), tune_get(TuneKey{TUNE_SIGMA, c, 1, 0}).kind == SIGMA_DQDS,
                                      P.img.add(tab), class_name(kSigmaNames, c)});
        }
        if (!scls.empty()) {
            double *msin = at<double>(ws, plan->msin_off);
            P.steps.push_back([=](const unsigned char *t, hipStream_t s) {
                const bool ready = fork_sigma && plan->ev_fork && plan->side[figaro_plan::kSide - 1] &&
                                   plan->ev_join[figaro_plan::kSide - 1];
                const int nb = ready ? std::min<int>((int)scls.size(), figaro_plan::kSide) : 1;
                if (nb > 1) HIPCHK(hipEventRecord(plan->ev_fork, s), "sigma fork");
                for (int k = 0; k < (int)scls.size(); k++) {
                    hipStream_t sk = nb > 1 ? plan->side[k % nb] : s;
                    if (nb > 1 && k < nb) HIPCHK(hipStreamWaitEvent(sk, plan->ev_fork, 0), "sigma fork wait");
                    const SigmaClass &e = scls[k];
                    Stage st(e.name, sk);
                    HIPCHK(launch_sigma_batch(e.c, R, sigma, (const int64_t *)(t + e.off), e.n, msin, sk, e.dqds),
                           "batched sigma");
                }
                for (int k = 0; k < nb && nb > 1; k++) {
                    HIPCHK(hipEventRecord(plan->ev_join[k], plan->side[k]), "sigma join");
                    HIPCHK(hipStreamWaitEvent(s, plan->ev_join[k], 0), "sigma join wait");
                }
                return FIGARO_OK;
            });
        }
    };
    bool refine_any = false;
    for (const Layout &L : plan->layouts) refine_any = refine_any || L.refine;
    std::vector<size_t> all, wide, rest;
    for (size_t i = 0; i < count; i++) {
        all.push_back(i);
        (sigma_width_class((int)plan->shapes[i].N()) == 128 ? wide : rest).push_back(i);
    }
    if (!refine_any && fuse_trees && plan->chains && !wide.empty() && !rest.empty()) {
        P.set_lane(1);
        emit_trees(wide, "tsqr_narrow");
        emit_roots(wide);
        emit_sigma(wide, false);
        P.set_lane(2);
        emit_trees(rest, "tsqr_narrow_b");
        emit_roots(rest);
        emit_sigma(rest, false);
        P.set_lane(0);
    } else {
        emit_trees(all, "tsqr_narrow");
        emit_roots(all);
    // refinement sweep of every instance (refined forms): the Gram blocks of all instances
    // in one tile launch and one reduce launch per input type, then one workgroup per
    // instance for the N x N part
    std::vector<GramJob> gjobs[2];
    std::vector<RefineSmall> smalls;
    for (size_t i = 0; i < count; i++) {
        const Shape &sh = plan->shapes[i];
        const Layout &L = plan->layouts[i];
        if (!L.refine) continue;
        void *lws = slice(i);
        const figaro_instance *in = &plan->inst[i];
        GramJob j3[3];
        gram_jobs(in->A.data, sh.in_f64, sh.lda, sh.m1, (int)sh.n1, in->B.data, sh.ldb, sh.m2, (int)sh.n2,
                  groups_of(lws, L), !sh.keyed, sh.two_sided ? at<double>(lws, L.headsA) : nullptr,
                  at<double>(lws, L.headsB), L.gcap, at<double>(lws, L.partial), at<double>(lws, L.gram), j3,
                  kBatchGramBlocks);
        for (const GramJob &J : j3) gjobs[sh.in_f64].push_back(J);
        const int N = (int)sh.N();
        smalls.push_back(RefineSmall{at<double>(lws, L.gram), at<double>(lws, L.rt), N, N, at<double>(lws, L.gy),
                                     at<int32_t>(lws, L.failed), R + plan->r_off[i], N});
    }
    for (int f = 0; f < 2; f++) {
        const std::vector<GramJob> &jobs = gjobs[f];
        if (jobs.empty()) continue;
        std::vector<int4> tiles;
        std::vector<int2> reds;
        for (int j = 0; j < (int)jobs.size(); j++) {
            const GramJob &J = jobs[j];
            for (int ti = 0; ti < J.gx; ti++)
                for (int tj = 0; tj < J.gy; tj++)
                    for (int c = 0; c < J.nch; c++)
                        if (J.mode != 0 || tj <= ti) tiles.push_back(make_int4(j, ti, tj, c));  // symmetric: lower tiles
            const int64_t out = (int64_t)J.nx * (J.mode == 0 ? J.nx : J.ny);
            for (int64_t b = 0; b < (out + 255) / 256; b++) reds.push_back(make_int2(j, (int)b));
        }
        const size_t jo = P.img.add(jobs), to = P.img.add(tiles), ro = P.img.add(reds);
        const int64_t nt = (int64_t)tiles.size(), nr = (int64_t)reds.size();
        P.steps.push_back([=](const unsigned char *t, hipStream_t s) {
            Stage st("refine_gram", s);
            HIPCHK(launch_gram_batch(f, (const GramJob *)(t + jo), (const int4 *)(t + to), nt, (const int2 *)(t + ro),
                                     nr, s),
                   "batched gram");
            return FIGARO_OK;
        });
    }
    if (!smalls.empty()) {
        const size_t off = P.img.add(smalls);
        const int n = (int)smalls.size();
        P.steps.push_back([=](const unsigned char *t, hipStream_t s) {
            Stage st("refine_solve", s);
            HIPCHK(launch_refine_small_batch((const RefineSmall *)(t + off), n, s), "batched refinement");
            return FIGARO_OK;
        });
    }

        emit_sigma(all, true);
    }
    P.set_lane(0);
    return P;
}

// The steps in order; a run of side-lane steps is forked from the launch stream (every
// side stream waits on it) and joined back before the next launch-stream step or the end.
// Without the plan's side streams every step runs on the launch stream.
int run_program(const Program &P, const unsigned char *tables, hipStream_t s)
{
    const figaro_plan *pl = P.plan;
    const bool side_ok = pl && pl->ev_fork && pl->side[figaro_plan::kSide - 1] && pl->ev_join[figaro_plan::kSide - 1];
    // only the side streams the program uses are forked and joined (no empty branches)
    int nside = 0;
    for (int l : P.lanes) nside = std::max(nside, std::min(l, (int)figaro_plan::kSide));
    bool forked = false;
    auto join = [&]() -> int {
        for (int k = 0; k < nside; k++) {
            HIPCHK(hipEventRecord(pl->ev_join[k], pl->side[k]), "join record");
            HIPCHK(hipStreamWaitEvent(s, pl->ev_join[k], 0), "join wait");
        }
        forked = false;
        return FIGARO_OK;
    };
    for (size_t i = 0; i < P.steps.size(); i++) {
        const int lane = i < P.lanes.size() ? P.lanes[i] : 0;
        hipStream_t st = s;
        if (lane > 0 && side_ok) {
            if (!forked) {
                HIPCHK(hipEventRecord(pl->ev_fork, s), "fork record");
                for (int k = 0; k < nside; k++)
                    HIPCHK(hipStreamWaitEvent(pl->side[k], pl->ev_fork, 0), "fork wait");
                forked = true;
            }
            st = pl->side[(lane - 1) % figaro_plan::kSide];
        } else if (forked) {
            int rc = join();
            if (rc) return rc;
        }
        int rc = P.steps[i](tables, st);
        if (rc) return rc;
    }
    if (forked) return join();
    return FIGARO_OK;
}

}  // namespace

extern "C" {

int figaro_plan_create(const figaro_instance *inst, int32_t count, int32_t precision,
                       figaro_plan **out)
{
    if (!inst || count < 1 || !out) return fail(FIGARO_EINVAL, "bad plan arguments");
    figaro_plan *p = new figaro_plan();
    size_t off = 0;
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
        Layout L = make_layout(sh, true);
        p->inst.push_back(inst[i]);
        p->shapes.push_back(sh);
        p->ws_off.push_back(off);
        off += align_up(L.total);
        p->layouts.push_back(std::move(L));
        p->r_off.push_back(p->r_total);
        p->s_off.push_back(p->s_total);
        p->r_total += sh.N() * sh.N();
        p->s_total += sh.N();
    }
    p->msin_off = off;
    p->chains = tune_get(TuneKey{TUNE_PLAN, p->shapes[0].precision == FIGARO_PLAIN_FP64, 1, 0}).kind != 0;
    // multisection inputs: 2 N + 2 doubles per instance
    p->ws_bytes = p->msin_off + align_up(sizeof(double) * (size_t)(2 * p->s_total + 2 * (int64_t)count));
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

namespace {

int plan_check(figaro_plan *plan, void *ws, size_t ws_bytes, double *R, double *sigma)
{
    if (!plan || !R || !sigma) return fail(FIGARO_EINVAL, "plan, R or sigma is NULL");
    if (!ws) return fail(FIGARO_EINVAL, "workspace is NULL");
    if (((uintptr_t)ws) % kAlign) return fail(FIGARO_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < plan->ws_bytes) return fail(FIGARO_EWORKSPACE, "workspace too small");
    return FIGARO_OK;
}

// The record of (ws, R, sigma); its launch tables (the image of `prog`) are uploaded on
// first use.
int plan_exec(figaro_plan *plan, void *ws, double *R, double *sigma, const Program &prog,
              figaro_plan::Exec **out)
{
    // the sigma stage's side streams and events, made on the first execution (a failed
    // attempt leaves the missing ones null and the stage on the launch stream alone)
    if (!plan->ev_fork) HIPCHK(hipEventCreateWithFlags(&plan->ev_fork, hipEventDisableTiming), "plan fork event");
    for (int k = 0; k < figaro_plan::kSide; k++) {
        if (!plan->side[k]) HIPCHK(hipStreamCreateWithFlags(&plan->side[k], hipStreamNonBlocking), "plan side stream");
        if (!plan->ev_join[k])
            HIPCHK(hipEventCreateWithFlags(&plan->ev_join[k], hipEventDisableTiming), "plan join event");
    }
    auto key = std::make_tuple(ws, R, sigma);
    auto it = plan->execs.find(key);
    if (it == plan->execs.end()) {
        figaro_plan::Exec ex;
        const size_t nb = prog.img.bytes.size();
        HIPCHK(hipMalloc((void **)&ex.tables, std::max<size_t>(nb, 1)), "plan launch tables");
        if (nb) {
            hipError_t e = hipMemcpy(ex.tables, prog.img.bytes.data(), nb, hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                (void)hipFree(ex.tables);
                return hip_fail(e, "plan launch tables");
            }
        }
        it = plan->execs.emplace(key, ex).first;
    }
    *out = &it->second;
    return FIGARO_OK;
}

}  // namespace

int figaro_plan_execute(figaro_plan *plan, void *ws, size_t ws_bytes, double *R, double *sigma,
                        void *stream)
{
    int rc = plan_check(plan, ws, ws_bytes, R, sigma);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    auto it = plan->execs.find(std::make_tuple(ws, R, sigma));
    if (it == plan->execs.end() || !it->second.graph) {
        const Program prog = build_program(plan, ws, R, sigma);
        figaro_plan::Exec *ex = nullptr;
        rc = plan_exec(plan, ws, R, sigma, prog, &ex);
        if (rc) return rc;
        if (!plan->cap_stream)
            HIPCHK(hipStreamCreateWithFlags(&plan->cap_stream, hipStreamNonBlocking), "plan stream");
        hipGraph_t graph = nullptr;
        HIPCHK(hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
        t_capturing = true;
        rc = run_program(prog, ex->tables, plan->cap_stream);
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
        ex->graph = exec;
        it = plan->execs.find(std::make_tuple(ws, R, sigma));
    }
    Stage st("plan_graph", s);
    HIPCHK(hipGraphLaunch(it->second.graph, s), "graph launch");
    return FIGARO_OK;
}

int figaro_plan_execute_eager(figaro_plan *plan, void *ws, size_t ws_bytes, double *R, double *sigma,
                              void *stream)
{
    int rc = plan_check(plan, ws, ws_bytes, R, sigma);
    if (rc) return rc;
    const Program prog = build_program(plan, ws, R, sigma);
    figaro_plan::Exec *ex = nullptr;
    rc = plan_exec(plan, ws, R, sigma, prog, &ex);
    if (rc) return rc;
    return run_program(prog, ex->tables, (hipStream_t)stream);
}

// ------------------------------------------------------------ autotuning
//
// For each class of narrow regions (same accumulation type and padded width) the
// candidates of the tuning table are timed on the caller's own problem: the launches
// run eagerly with stage events (one warm-up, then three timed runs), the class's tree
// stage is read, and the fastest candidate becomes the table entry of every row count the
// class holds.  Tuning allocates (launch tables) and synchronises; it changes neither
// workspace sizes nor results beyond rounding order.
}  // extern "C"

namespace {

struct TimingGuard {
    bool was;
    TimingGuard() : was(g_timing.on.load()) { g_timing.on.store(true); }
    ~TimingGuard() { g_timing.on.store(was); }
};

// Milliseconds of the recorded stages accepted by `want`, summed; every record is consumed.
template <typename F>
int take_stage_ms(F want, double *ms)
{
    std::lock_guard<std::mutex> lk(g_timing.mu);
    double tot = 0.0;
    for (auto &r : g_timing.recs) {
        hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess) return hip_fail(e, "tuning sync");
        float t = 0.f;
        e = hipEventElapsedTime(&t, r.a, r.b);
        if (e != hipSuccess) return hip_fail(e, "tuning elapsed");
        if (want(r.name)) tot += t;
        g_timing.pool.push_back(r.a);
        g_timing.pool.push_back(r.b);
    }
    g_timing.recs.clear();
    *ms = tot;
    return FIGARO_OK;
}

constexpr int kTuneReps = 3;

// The caller may still have a launch of one of these graphs (or an eager execution that
// reads these tables) in flight on any stream: the device is drained before they go.
void plan_drop_execs(figaro_plan *plan)
{
    if (plan->execs.empty()) return;
    (void)hipDeviceSynchronize();
    for (auto &kv : plan->execs) {
        if (kv.second.graph) (void)hipGraphExecDestroy(kv.second.graph);
        if (kv.second.tables) (void)hipFree(kv.second.tables);
    }
    plan->execs.clear();
}

// New layouts from the tuning table.  The cached launch tables and graphs were built for
// the old ones (tree sizes, leaf counts), so they go too.
void plan_relayout(figaro_plan *plan)
{
    plan_drop_execs(plan);
    for (size_t i = 0; i < plan->inst.size(); i++) plan->layouts[i] = make_layout(plan->shapes[i], true);
}

}  // namespace

extern "C" {

int figaro_plan_autotune(figaro_plan *plan, void *ws, size_t ws_bytes, double *R, double *sigma, void *stream)
{
    int rc = plan_check(plan, ws, ws_bytes, R, sigma);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int acc = plan->shapes[0].precision == FIGARO_PLAIN_FP64;
    // classes: padded width -> the row counts (log2) of its regions
    std::map<int, std::vector<int>> cls;
    for (const Layout &L : plan->layouts)
        for (const Region &r : L.regions)
            if (r.wave && !r.skip && r.rows_cap > 0) cls[r.np].push_back(rows_log2(r.rows_cap));
    plan_drop_execs(plan);
    TimingGuard tg;
    // time of `stage` (summed over kTuneReps runs after a warm-up) with candidate `cand` for
    // the tuning key `key`, the trees of each class in their own launch or all in one
    auto time_cand = [&](const TuneKey &key, const TreeTune &cand, bool fused, const char *stage, double *ms) {
        tune_override(&key, &cand);
        plan_relayout(plan);
        const Program prog = build_program(plan, ws, R, sigma, fused);
        figaro_plan::Exec *ex = nullptr;
        int e = plan_exec(plan, ws, R, sigma, prog, &ex);
        if (!e) e = run_program(prog, ex->tables, s);  // warm-up
        double t = 0.0;
        if (!e) e = take_stage_ms([](const char *) { return false; }, &t);
        for (int i = 0; i < kTuneReps && !e; i++) e = run_program(prog, ex->tables, s);
        *ms = 0.0;
        if (!e) e = take_stage_ms([stage](const char *n) { return std::strcmp(n, stage) == 0; }, ms);
        plan_drop_execs(plan);
        tune_override(nullptr, nullptr);
        return e;
    };
    // each class alone
    for (auto &kv : cls) {
        const int np = kv.first;
        const TuneKey key{acc, np, 1, 0};
        double best_ms = 1e300;
        TreeTune best = tune_default(key);
        for (const TreeTune &cand : tune_candidates(key)) {
            double ms = 0.0;
            rc = time_cand(key, cand, false, class_name(kTreeNames, np), &ms);
            if (rc) {
                plan_relayout(plan);
                return rc;
            }
            if (ms < best_ms) {
                best_ms = ms;
                best = cand;
            }
        }
        for (int l : kv.second) tune_set(TuneKey{acc, np, 1, l}, best, best_ms / kTuneReps);
    }
    // then the classes together: a plan runs every narrow width in one launch, where the
    // balance of the leaves over the compute units sets the time -- one pass of coordinate
    // descent over the classes, widest first, on the shared launch (chains are not tuned:
    // a plan runs them as the tuning table says, one after the other by default)
    if (std::count_if(cls.begin(), cls.end(), [](const auto &kv) { return kv.first <= 64; }) > 1) {
        for (auto it = cls.rbegin(); it != cls.rend(); ++it) {
            const int np = it->first;
            if (np > 64) continue;  // not in the shared launch
            const TuneKey key{acc, np, 1, 0};
            double best_ms = 1e300;
            TreeTune best = tune_get(TuneKey{acc, np, 1, it->second.front()});
            for (const TreeTune &cand : tune_candidates(key)) {
                double ms = 0.0;
                rc = time_cand(key, cand, true, "tsqr_narrow", &ms);
                if (rc) {
                    plan_relayout(plan);
                    return rc;
                }
                if (ms < best_ms) {
                    best_ms = ms;
                    best = cand;
                }
            }
            for (int l : it->second) tune_set(TuneKey{acc, np, 1, l}, best, best_ms / kTuneReps);
        }
    }
    plan_relayout(plan);
    // sigma route per width class (multisection or dqds after the bidiagonalisation)
    std::vector<int> scls;
    for (const Shape &sh : plan->shapes) {
        const int c = sigma_width_class((int)sh.N());
        if (c && std::find(scls.begin(), scls.end(), c) == scls.end()) scls.push_back(c);
    }
    for (int c : scls) {
        const TuneKey key{TUNE_SIGMA, c, 1, 0};
        const char *stage = class_name(kSigmaNames, c);
        double best_ms = 1e300;
        TreeTune best = tune_default(key);
        for (const TreeTune &cand : tune_candidates(key)) {
            tune_override(&key, &cand);
            const Program prog = build_program(plan, ws, R, sigma);
            figaro_plan::Exec *ex = nullptr;
            rc = plan_exec(plan, ws, R, sigma, prog, &ex);
            if (!rc) rc = run_program(prog, ex->tables, s);
            double ms = 0.0;
            if (!rc) rc = take_stage_ms([](const char *) { return false; }, &ms);
            for (int i = 0; i < kTuneReps && !rc; i++) rc = run_program(prog, ex->tables, s);
            if (!rc) rc = take_stage_ms([stage](const char *n) { return std::strcmp(n, stage) == 0; }, &ms);
            plan_drop_execs(plan);
            if (rc) {
                tune_override(nullptr, nullptr);
                return rc;
            }
            if (ms < best_ms) {
                best_ms = ms;
                best = cand;
            }
        }
        tune_override(nullptr, nullptr);
        tune_set(key, best, best_ms / kTuneReps);
    }
    return FIGARO_OK;
}

int figaro_r_autotune(const figaro_table *A, const figaro_table *B, int32_t precision, double *R, int64_t ldr,
                      void *ws, size_t ws_bytes, void *stream)
{
    Shape sh;
    int rc = make_shape(A, B, precision, &sh);
    if (rc) return rc;
    if (!R) return fail(FIGARO_EINVAL, "R is NULL");
    if (ldr < sh.N()) return fail(FIGARO_EINVAL, "ldr < n1 + n2");
    Layout L0 = make_layout(sh);
    rc = check_ws(L0, ws, ws_bytes);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int acc = sh.precision == FIGARO_PLAIN_FP64;
    std::map<int, std::vector<int>> cls;
    for (const Region &r : L0.regions)
        if (r.wave && !r.skip && r.rows_cap > 0) cls[r.np].push_back(rows_log2(r.rows_cap));
    TimingGuard tg;
    auto is_tree = [](const char *n) { return std::strncmp(n, "tsqr_", 5) == 0 && std::strcmp(n, "tsqr_root") != 0; };
    for (auto &kv : cls) {
        const int np = kv.first;
        const TuneKey key{acc, np, 0, 0};
        double best_ms = 1e300;
        TreeTune best = tune_default(key);
        for (const TreeTune &cand : tune_candidates(key)) {
            tune_override(&key, &cand);
            const Layout L = make_layout(sh);
            double ms = 0.0;
            rc = run_r(A, B, sh, L, R, ldr, ws, s);
            if (!rc) rc = take_stage_ms([](const char *) { return false; }, &ms);
            for (int i = 0; i < kTuneReps && !rc; i++) rc = run_r(A, B, sh, L, R, ldr, ws, s);
            if (!rc) rc = take_stage_ms(is_tree, &ms);
            if (rc) {
                tune_override(nullptr, nullptr);
                return rc;
            }
            if (ms < best_ms) {
                best_ms = ms;
                best = cand;
            }
        }
        tune_override(nullptr, nullptr);
        for (int l : kv.second) tune_set(TuneKey{acc, np, 0, l}, best, best_ms / kTuneReps);
    }
    return FIGARO_OK;
}

int figaro_tune_load(const char *path)
{
    if (!path) return fail(FIGARO_EINVAL, "path is NULL");
    const int n = tune_load(path);
    if (n < 0) return fail(FIGARO_EINVAL, std::string("cannot read tuning cache ") + path);
    return FIGARO_OK;
}

int figaro_tune_save(const char *path)
{
    if (!path) return fail(FIGARO_EINVAL, "path is NULL");
    if (tune_save(path) != 0) return fail(FIGARO_EINVAL, std::string("cannot write tuning cache ") + path);
    return FIGARO_OK;
}

int figaro_tune_dump(char *buf, size_t cap, size_t *len)
{
    const std::string d = tune_dump();
    if (len) *len = d.size();
    if (buf && cap > 0) {
        const size_t n = std::min(cap - 1, d.size());
        std::memcpy(buf, d.data(), n);
        buf[n] = 0;
    }
    return FIGARO_OK;
}

void figaro_plan_destroy(figaro_plan *plan)
{
    if (!plan) return;
    plan_drop_execs(plan);
    if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);
    for (int k = 0; k < figaro_plan::kSide; k++) {
        if (plan->side[k]) (void)hipStreamDestroy(plan->side[k]);
        if (plan->ev_join[k]) (void)hipEventDestroy(plan->ev_join[k]);
    }
    if (plan->ev_fork) (void)hipEventDestroy(plan->ev_fork);
    delete plan;
}

}  // extern "C"
