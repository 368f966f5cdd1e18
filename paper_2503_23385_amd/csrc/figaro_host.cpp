// Host runtime of the gfx950 Figaro library: argument checks, workspace
// layout, and the launch sequence behind the C ABI of include/figaro.h.
//
// The pipeline follows the paper's Figaro-GPU steps (Experiments section):
// heads/tails of B per key group, the compact matrix of Claim 1, a
// Householder QR of that matrix for R, and the singular values of R.  The
// differences are in how each step runs on the device: a segmented scan with
// look-back instead of one thread per column, no row/column-major transpose,
// and a TSQR reduction instead of a library QR.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
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

struct TimingRec {
    const char *name;
    hipEvent_t a, b;
};

struct Timing {
    bool on = false;
    std::vector<TimingRec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t get()
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

// Brackets the launches of one stage with events when timing is on.
struct Stage {
    const char *name;
    hipStream_t s;
    hipEvent_t a = nullptr;
    Stage(const char *n, hipStream_t st) : name(n), s(st)
    {
        if (g_timing.on) {
            a = g_timing.get();
            if (a) (void)hipEventRecord(a, s);
        }
    }
    ~Stage()
    {
        if (a) {
            hipEvent_t b = g_timing.get();
            if (b) {
                (void)hipEventRecord(b, s);
                g_timing.recs.push_back({name, a, b});
            } else {
                g_timing.pool.push_back(a);
            }
        }
    }
};

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Shape {
    int64_t m1, n1, lda, m2, n2, ldb;
    int in_f64;
    bool keyed;
    int precision;
    int64_t N() const { return n1 + n2; }
};

// TSQR reduction plan for one region: leaves, then levels of the tree.
struct TreePlan {
    int np = 0, width = 0, col_off = 0;
    int leaves = 0;
    std::vector<int> levels;  // workgroups per level after the leaves
    int final_count = 0;      // triangles entering the root
};

struct Layout {
    size_t status, counts, ticket;
    size_t blkA, blkB, runA, runB, matchA, blkM, blkS;
    size_t g[7];
    int64_t gcap;
    size_t heads, tileF, tileS, carry;
    size_t M1, M2;
    int m_f64;
    size_t triA[2], triB[2];
    size_t rtmp;
    size_t total;
    ScanPlan sp;
    TreePlan ta, tb;
    int np_root;
    int nbA, nbB;
};

constexpr int kTreeArity = 2;
constexpr int kRootMax = 2;
constexpr int kMaxLeaves = 4096;

TreePlan plan_tree(int64_t rows_upper, int width, int col_off, int np_root_acc)
{
    (void)np_root_acc;
    TreePlan t;
    t.np = tsqr_padded_width(width);
    t.width = width;
    t.col_off = col_off;
    const int br = tsqr_block_rows(t.np);
    const int64_t per_wg = std::max<int64_t>(2 * (int64_t)width, 4 * (int64_t)br);
    int64_t leaves = (rows_upper + per_wg - 1) / per_wg;
    leaves = std::max<int64_t>(1, std::min<int64_t>(leaves, kMaxLeaves));
    t.leaves = (int)leaves;
    int cur = t.leaves;
    while (cur > kRootMax) {
        cur = (cur + kTreeArity - 1) / kTreeArity;
        t.levels.push_back(cur);
    }
    t.final_count = cur;
    return t;
}

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
    if (precision != FIGARO_PLAIN_FP64 && precision != FIGARO_MIXED_FP32 &&
        precision != FIGARO_MIXED_FP32_REFINE)
        return fail(FIGARO_EINVAL, "unknown precision");
    const int64_t N = A->cols + B->cols;
    if (N > FIGARO_MAX_N) return fail(FIGARO_EINVAL, "n1 + n2 exceeds FIGARO_MAX_N");
    // Widths this build's TSQR kernels accept.
    const bool fp64_acc = precision == FIGARO_PLAIN_FP64;
    const int np = tsqr_padded_width((int)N);
    if (np == 0 || (fp64_acc && np > 128))
        return fail(FIGARO_EINVAL, "n1 + n2 wider than this build supports for the chosen precision");
    if (B->cols > 512) return fail(FIGARO_EINVAL, "n2 > 512");
    sh->m1 = A->rows;
    sh->n1 = A->cols;
    sh->lda = A->ld;
    sh->m2 = B->rows;
    sh->n2 = B->cols;
    sh->ldb = B->ld;
    sh->in_f64 = A->dtype == FIGARO_F64;
    sh->keyed = A->keys != nullptr;
    sh->precision = precision;
    return FIGARO_OK;
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
    L.ticket = take(sizeof(int32_t) * 4);
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
    L.heads = take(sizeof(double) * L.gcap * s.n2);
    L.m_f64 = s.precision == FIGARO_PLAIN_FP64;
    const size_t esz = L.m_f64 ? 8 : 4;
    L.sp = scan_plan(s.m2, s.n2, s.in_f64 ? 8 : 4);
    L.tileF = take(sizeof(int32_t) * std::max<int64_t>(1, L.sp.ntiles));
    L.tileS = take(sizeof(double) * std::max<int64_t>(1, L.sp.ntiles) * s.n2);
    L.carry = take(sizeof(double) * std::max<int64_t>(1, L.sp.ntiles) * s.n2);
    const int64_t N = s.N();
    L.M1 = take(esz * std::max<int64_t>(1, s.m1) * N);
    L.M2 = take(esz * std::max<int64_t>(1, s.m2 - 1) * s.n2);
    L.ta = plan_tree(s.m1, (int)N, 0, 0);
    L.tb = plan_tree(std::max<int64_t>(0, s.m2 - 1), (int)s.n2, (int)s.n1, 0);
    L.np_root = L.ta.np;
    const size_t triA_sz = sizeof(double) * (size_t)L.ta.leaves * N * L.ta.np;
    const size_t triA2_sz = sizeof(double) * (size_t)(L.ta.levels.empty() ? 1 : L.ta.levels[0]) * N * L.ta.np;
    const size_t triB_sz = sizeof(double) * (size_t)L.tb.leaves * s.n2 * L.tb.np;
    const size_t triB2_sz = sizeof(double) * (size_t)(L.tb.levels.empty() ? 1 : L.tb.levels[0]) * s.n2 * L.tb.np;
    L.triA[0] = take(triA_sz);
    L.triA[1] = take(triA2_sz);
    L.triB[0] = take(triB_sz);
    L.triB[1] = take(triB2_sz);
    L.rtmp = take(sizeof(double) * N * L.np_root);
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

#define HIPCHK(expr, where)                          \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

int run_compact(const figaro_table *A, const figaro_table *B, const Shape &sh, const Layout &L,
                void *ws, hipStream_t s)
{
    Groups g = groups_of(ws, L);
    int32_t *status = at<int32_t>(ws, L.status);
    Stage st_group("group", s);
    HIPCHK(launch_group_init(status, g.counts, nullptr, nullptr, 0, s), "init");
    if (sh.keyed) {
        HIPCHK(launch_group_keys(A->keys, sh.m1, B->keys, sh.m2, g, at<int32_t>(ws, L.blkA),
                                 at<int32_t>(ws, L.blkB), at<int32_t>(ws, L.runA),
                                 at<int32_t>(ws, L.runB), at<int32_t>(ws, L.matchA),
                                 at<int32_t>(ws, L.blkM), at<int64_t>(ws, L.blkS), status, s),
               "grouping");
    } else {
        HIPCHK(launch_group_cartesian(g, sh.m1, sh.m2, s), "grouping");
    }
    double *heads = at<double>(ws, L.heads);
    {
    Stage st("scan", s);
    HIPCHK(launch_seg_scan(B->data, sh.in_f64, sh.ldb, sh.m2, sh.n2, g, !sh.keyed,
                           at<void>(ws, L.M2), L.m_f64, heads, at<int32_t>(ws, L.tileF),
                           at<double>(ws, L.tileS), at<double>(ws, L.carry), L.sp, s),
           "head/tail scan");
    }
    Stage st_asm("assemble", s);
    HIPCHK(launch_assemble_a(A->data, sh.in_f64, sh.lda, sh.m1, sh.n1, sh.n2, g, !sh.keyed, heads,
                             at<void>(ws, L.M1), L.m_f64, s),
           "region-1 assembly");
    return FIGARO_OK;
}

// Run one region's leaves and tree levels; returns the buffer holding its final triangles.
int run_tree(const TreePlan &t, RowSrc leaf_src, int acc_f64_leaf, int acc_f64_tree, int in_f64,
             void *ws, const size_t bufs[2], double **final_buf, const char *leaf_name, hipStream_t s)
{
    RowSrc none{};
    double *cur = at<double>(ws, bufs[0]);
    const int64_t stride = (int64_t)t.width * t.np;
    {
        Stage st(leaf_name, s);
        HIPCHK(launch_tsqr_stream(t.np, acc_f64_leaf, in_f64, leaf_src, none, 1, t.width, 0, t.leaves,
                                  cur, stride, s),
               "tsqr leaves");
    }
    int count = t.leaves;
    int which = 0;
    for (int nwg : t.levels) {
        double *nxt = at<double>(ws, bufs[which ^ 1]);
        RowSrc src{cur, nullptr, (int64_t)count * t.width, t.np, 0, t.width};
        Stage st("tsqr_tree", s);
        HIPCHK(launch_tsqr_stream(t.np, acc_f64_tree, 1, src, none, 1, t.width, t.width, nwg, nxt,
                                  stride, s),
               "tsqr tree");
        cur = nxt;
        which ^= 1;
        count = nwg;
    }
    *final_buf = cur;
    return FIGARO_OK;
}

int run_r(const figaro_table *A, const figaro_table *B, const Shape &sh, const Layout &L, double *R,
          int64_t ldr, void *ws, hipStream_t s)
{
    int rc = run_compact(A, B, sh, L, ws, s);
    if (rc) return rc;
    Groups g = groups_of(ws, L);
    const int N = (int)sh.N();
    const int acc_leaf = sh.precision == FIGARO_PLAIN_FP64;
    const int acc_tree = acc_leaf;
    RowSrc srcA{at<void>(ws, L.M1), g.counts + CNT_R1, 0, N, 0, N};
    RowSrc srcB{at<void>(ws, L.M2), g.counts + CNT_R2, 0, sh.n2, 0, (int)sh.n2};
    double *fa = nullptr, *fb = nullptr;
    rc = run_tree(L.ta, srcA, acc_leaf, acc_tree, L.m_f64, ws, L.triA, &fa, "tsqr_leaf_m1", s);
    if (rc) return rc;
    rc = run_tree(L.tb, srcB, acc_leaf, acc_tree, L.m_f64, ws, L.triB, &fb, "tsqr_leaf_m2", s);
    if (rc) return rc;
    // Root: [R_1 ; 0 | R_2] -> R in FP64.
    RowSrc ra{fa, nullptr, (int64_t)L.ta.final_count * N, L.ta.np, 0, N};
    RowSrc rb{fb, nullptr, (int64_t)L.tb.final_count * sh.n2, L.tb.np, (int)sh.n1, (int)sh.n2};
    double *rt = at<double>(ws, L.rtmp);
    {
        Stage st("tsqr_root", s);
        HIPCHK(launch_tsqr_stream(L.np_root, 1, 1, ra, rb, 2, N, 0, 1, rt, (int64_t)N * L.np_root, s),
               "tsqr root");
    }
    Stage st("sign", s);
    HIPCHK(launch_sign_normalise(rt, 1, L.np_root, N, R, ldr, s), "sign normalisation");
    return FIGARO_OK;
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
    out->heads = at<double>(ws, L.heads);
    out->m1 = at<void>(ws, L.M1);
    out->m2 = at<void>(ws, L.M2);
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
    *bytes = kAlign;
    return FIGARO_OK;
}

int figaro_sigma(const double *R, int64_t n, int64_t ldr, double *sigma, void *ws, size_t ws_bytes,
                 void *stream)
{
    if (n < 1 || n > FIGARO_MAX_N) return fail(FIGARO_EINVAL, "n out of range");
    if (!R || !sigma) return fail(FIGARO_EINVAL, "R or sigma is NULL");
    if (ldr < n) return fail(FIGARO_EINVAL, "ldr < n");
    if (!ws) return fail(FIGARO_EINVAL, "workspace is NULL");
    if (ws_bytes < kAlign) return fail(FIGARO_EWORKSPACE, "workspace too small");
    if (n > 128) return fail(FIGARO_EINVAL, "n > 128 is not supported by this build's Jacobi");
    Stage st("jacobi", (hipStream_t)stream);
    hipError_t e = launch_jacobi(R, (int)n, ldr, sigma, 60, (int32_t *)ws, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "jacobi");
    return FIGARO_OK;
}

int figaro_timing_enable(int32_t on)
{
    g_timing.on = on != 0;
    return FIGARO_OK;
}

int figaro_timing_read(const char **names, double *ms, int32_t *launches, int32_t cap,
                       int32_t *count)
{
    if (!count) return fail(FIGARO_EINVAL, "count is NULL");
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

// ------------------------------------------------------------------ plans

}  // extern "C"

struct figaro_plan {
    std::vector<figaro_instance> inst;
    std::vector<Shape> shapes;
    std::vector<Layout> layouts;
    std::vector<int64_t> r_off, s_off;
    int64_t r_total = 0, s_total = 0;
    int precision = 0;
    size_t ws_bytes = 0;
    size_t sig_ws = 0;
};

extern "C" {

int figaro_plan_create(const figaro_instance *inst, int32_t count, int32_t precision,
                       figaro_plan **out)
{
    if (!inst || count < 1 || !out) return fail(FIGARO_EINVAL, "bad plan arguments");
    figaro_plan *p = new figaro_plan();
    p->precision = precision;
    size_t wsmax = 0;
    for (int i = 0; i < count; i++) {
        Shape sh;
        int rc = make_shape(&inst[i].A, &inst[i].B, precision, &sh);
        if (rc) {
            delete p;
            return rc;
        }
        Layout L = make_layout(sh);
        p->inst.push_back(inst[i]);
        p->shapes.push_back(sh);
        p->layouts.push_back(L);
        p->r_off.push_back(p->r_total);
        p->s_off.push_back(p->s_total);
        p->r_total += sh.N() * sh.N();
        p->s_total += sh.N();
        wsmax = std::max(wsmax, L.total);
    }
    p->ws_bytes = wsmax;
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
    for (size_t i = 0; i < plan->inst.size(); i++) {
        const Shape &sh = plan->shapes[i];
        const int64_t N = sh.N();
        int rc = run_r(&plan->inst[i].A, &plan->inst[i].B, sh, plan->layouts[i], R + plan->r_off[i], N,
                       ws, s);
        if (rc) return rc;
        Stage st("jacobi", s);
        hipError_t e = launch_jacobi(R + plan->r_off[i], (int)N, N, sigma + plan->s_off[i], 60,
                                     nullptr, s);
        if (e != hipSuccess) return hip_fail(e, "jacobi");
    }
    return FIGARO_OK;
}

void figaro_plan_destroy(figaro_plan *plan) { delete plan; }

}  // extern "C"
