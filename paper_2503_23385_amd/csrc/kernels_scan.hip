// Per-group QR head and tail of B, and assembly of region 1 of the compact
// matrix ("Figaro on GPUs: Two Tables", Section 1: the head operator
// H(B) = (1/sqrt m) sum_i B_i, the tail operator
// T(B)_i = (sqrt(i) B_{i+1} - S_i / sqrt(i)) / sqrt(i+1) with S_i the sum of the
// first i rows, and Claim 1's compact form).
//
// Head/tail: a segmented column scan of B (sums restart at every group start),
// accumulated in FP64 whatever the input or storage type.  Three launches:
//   1. tile reduce: each tile of rows produces its segmented aggregate
//      (F = "a group starts in the tile", S = column sums since the last start);
//   2. carry scan: one workgroup per column scans the tile aggregates in a fixed
//      order and writes, per tile, the sums carried into its first (continuing) group;
//   3. tile write: each tile rescans its rows with the carry and writes tail
//      row i of group g to region-2 row r2_g + i - 1, scaled by sqrt(m1_g), and
//      the head of a group that ends in the tile to heads[g].
// Every sum is formed in the same order on every run (no atomics, no
// timing-dependent look-back), so results are bitwise reproducible.  The
// second read of B is served by the Infinity Cache when B fits in it.
//
// Region 1: row r of A in group g becomes [sqrt(m2_g) A_r | H(B_g)] at row
// r1_g + (r - offA_g).
#include "common.h"

namespace figaro {
namespace {

constexpr int kScanThreads = 256;
constexpr int kMaxTileRows = 512;
constexpr int kMaxCols = 512;
constexpr int kCarryThreads = 1024;
constexpr int kBatchCarryThreads = 1024;  // 64 columns x 16 chunks of tiles (batched carry scan)

template <typename T>
__device__ inline double to_f64(T v) { return (double)v; }

// Last group index in [lo, hi) whose start <= s (starts ascending); lo if none.
__device__ inline int last_start_le(const int32_t *start, int lo, int hi, int64_t s)
{
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= s) lo = mid;
        else hi = mid;
    }
    return lo;
}

// First group index in [0, G) whose end (start + size) > s; G if none.
__device__ inline int first_end_gt(const int32_t *start, const int32_t *size, int G, int64_t s)
{
    int lo = 0, hi = G;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((int64_t)start[mid] + size[mid] > s) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// One tile of a table's rows: reduce (WRITE = false) or write tails/heads (WRITE = true).
// The tiles of two jobs (the two tables of the two-sided form) share one launch: blocks
// [0, j0.ntiles) take job 0, the rest job 1.
// Tile t of job J (its table's rows, group table J.g).
template <typename Tin, typename Tout, int CPT, int RPT, bool WRITE>
__device__ __forceinline__ void seg_tile(const ScanJob &J, const int t)
{
    const Groups g = J.g;
    const int cartesian = J.cartesian;
    const Tin *__restrict__ B = (const Tin *)J.in;
    const int64_t ldb = J.ld;
    const int m2 = J.m, n2 = J.n, Q = J.q;
    const ScanSide side = J.side;
    Tout *__restrict__ M2 = (Tout *)J.out;
    double *__restrict__ heads = J.heads;
    int32_t *__restrict__ tileF = J.tileF;
    double *__restrict__ tileS = J.tileS;
    const double *__restrict__ carry = J.carry;
    const int tid = threadIdx.x;
    const int ncolthr = (n2 + CPT - 1) / CPT;
    const int c = tid % ncolthr;
    const int q = tid / ncolthr;
    const bool active = q < Q;
    const int TR = Q * RPT;
    const int64_t t0 = (int64_t)t * TR;
    const int G = (int)g.counts[CNT_G];

    __shared__ int s_g0;
    __shared__ int m_g[kMaxTileRows], m_pos[kMaxTileRows], m_out[kMaxTileRows];
    __shared__ double m_c1[kMaxTileRows], m_c2[kMaxTileRows], m_hs[kMaxTileRows];
    __shared__ int a_f[kScanThreads];
    __shared__ double a_s[kMaxCols];

    // The tile's loads are issued first; they stay in flight during the metadata search.
    // Each load is unconditional, with the row and column clamped into the table (a
    // conditional load compiles to a branch that waits for it in turn).  Entries outside
    // the table are never used: their rows belong to no group and their columns are
    // never stored.
    double x[RPT][CPT];
#pragma unroll
    for (int i = 0; i < RPT; i++) {
        const int64_t s = t0 + (int64_t)q * RPT + i;
        const int64_t sc = s < m2 ? s : m2 - 1;
#pragma unroll
        for (int cc = 0; cc < CPT; cc++) {
            const int col = c + cc * ncolthr;
            x[i][cc] = to_f64(B[sc * ldb + (col < n2 ? col : n2 - 1)]);
        }
    }

    if (tid == 0) s_g0 = cartesian ? 0 : first_end_gt(side.off, side.size, G, t0);
    __syncthreads();
    const int g0 = s_g0;
    for (int r = tid; r < TR; r += kScanThreads) {
        const int64_t s = t0 + r;
        int gi = -1, pos = 0;
        if (s < m2 && G > 0) {
            if (cartesian) {
                gi = 0;
                pos = (int)s;
            } else if (g0 < G) {
                const int hi = min(G, g0 + r + 1);
                const int cand = last_start_le(side.off, g0, hi, s);
                if (side.off[cand] <= s && s < (int64_t)side.off[cand] + side.size[cand]) {
                    gi = cand;
                    pos = (int)(s - side.off[cand]);
                }
            }
        }
        m_g[r] = gi;
        m_pos[r] = pos;
        if (WRITE && gi >= 0) {
            const double sm1 = sqrt((double)side.other[gi]);
            const int m2g = side.size[gi];
            m_out[r] = side.obase[gi] - (side.sub_g ? gi : 0) + pos - 1;
            if (pos > 0) {
                const double sp = sqrt((double)pos), sp1 = sqrt((double)pos + 1.0);
                m_c1[r] = sm1 * sp / sp1;
                m_c2[r] = sm1 / (sp * sp1);
            }
            m_hs[r] = (pos == m2g - 1) ? 1.0 / sqrt((double)m2g) : 0.0;
        }
    }
    __syncthreads();

    // Thread aggregate over its rows: (f, s), f = "a segment starts in these rows".
    int f = 0;
    double sacc[CPT];
#pragma unroll
    for (int cc = 0; cc < CPT; cc++) sacc[cc] = 0.0;
    if (active) {
#pragma unroll
        for (int i = 0; i < RPT; i++) {
            const int lr = q * RPT + i;
            const int gi = m_g[lr];
            if (gi < 0 || m_pos[lr] == 0) {
                f = 1;
#pragma unroll
                for (int cc = 0; cc < CPT; cc++) sacc[cc] = (gi < 0) ? 0.0 : x[i][cc];
            } else {
#pragma unroll
                for (int cc = 0; cc < CPT; cc++) sacc[cc] += x[i][cc];
            }
        }
        if (c == 0) a_f[q] = f;
#pragma unroll
        for (int cc = 0; cc < CPT; cc++) {
            const int col = c + cc * ncolthr;
            if (col < n2) a_s[q * n2 + col] = sacc[cc];
        }
    }
    __syncthreads();

    // Exclusive prefix over earlier row groups (e) and the tile aggregate (F, S).
    int ef = 0, F = 0;
    double es[CPT], S[CPT];
#pragma unroll
    for (int cc = 0; cc < CPT; cc++) { es[cc] = 0.0; S[cc] = 0.0; }
    if (active) {
        for (int qq = 0; qq < Q; qq++) {
            const int af = a_f[qq];
#pragma unroll
            for (int cc = 0; cc < CPT; cc++) {
                const int col = c + cc * ncolthr;
                const double as = col < n2 ? a_s[qq * n2 + col] : 0.0;
                if (qq < q) es[cc] = af ? as : es[cc] + as;
                S[cc] = af ? as : S[cc] + as;
            }
            if (qq < q) ef |= af;
            F |= af;
        }
    }

    if (!WRITE) {
        if (active && q == 0) {
#pragma unroll
            for (int cc = 0; cc < CPT; cc++) {
                const int col = c + cc * ncolthr;
                if (col < n2) tileS[(int64_t)t * n2 + col] = S[cc];
            }
            if (c == 0) tileF[t] = F;
        }
        return;
    }

    // Second pass: tails and heads with the running FP64 prefix.
    if (!active) return;
    const bool need = m_g[0] >= 0 && m_pos[0] > 0;  // tile starts inside a group
    double run[CPT];
#pragma unroll
    for (int cc = 0; cc < CPT; cc++) {
        const int col = c + cc * ncolthr;
        const double cin = (need && col < n2) ? carry[(int64_t)t * n2 + col] : 0.0;
        run[cc] = (ef ? 0.0 : cin) + es[cc];
    }
#pragma unroll
    for (int i = 0; i < RPT; i++) {
        const int lr = q * RPT + i;
        const int gi = m_g[lr];
        if (gi < 0) {
#pragma unroll
            for (int cc = 0; cc < CPT; cc++) run[cc] = 0.0;
            continue;
        }
        const int pos = m_pos[lr];
        if (pos == 0) {
#pragma unroll
            for (int cc = 0; cc < CPT; cc++) run[cc] = 0.0;
        } else {
            const double c1 = m_c1[lr], c2 = m_c2[lr];
            Tout *out = M2 + (int64_t)m_out[lr] * n2;
#pragma unroll
            for (int cc = 0; cc < CPT; cc++) {
                const int col = c + cc * ncolthr;
                if (col < n2) out[col] = (Tout)(c1 * x[i][cc] - c2 * run[cc]);
            }
        }
#pragma unroll
        for (int cc = 0; cc < CPT; cc++) run[cc] += x[i][cc];
        const double hs = m_hs[lr];
        if (hs != 0.0) {
#pragma unroll
            for (int cc = 0; cc < CPT; cc++) {
                const int col = c + cc * ncolthr;
                if (col < n2) heads[(int64_t)gi * n2 + col] = run[cc] * hs;
            }
        }
    }
}

// The tiles of up to two inline jobs (the two tables of the two-sided form) in one
// launch: blocks [0, j0.ntiles) take job 0, the rest job 1.
template <typename Tin, typename Tout, int CPT, int RPT, bool WRITE>
__global__ __launch_bounds__(kScanThreads) void k_seg_tile(ScanJob j0, ScanJob j1)
{
    const bool second = (int64_t)blockIdx.x >= j0.ntiles;
    seg_tile<Tin, Tout, CPT, RPT, WRITE>(second ? j1 : j0, (int)(blockIdx.x - (second ? j0.ntiles : 0)));
}

// The tiles of a batch of jobs (device table): block b takes tile map[b].y of job map[b].x.
template <typename Tin, typename Tout, int CPT, int RPT, bool WRITE>
__global__ __launch_bounds__(kScanThreads) void k_seg_tile_batch(const ScanJob *__restrict__ jobs,
                                                                 const int2 *__restrict__ map)
{
    const int2 e = map[blockIdx.x];
    const ScanJob J = jobs[e.x];
    seg_tile<Tin, Tout, CPT, RPT, WRITE>(J, e.y);
}

// Exclusive segmented scan of the tile aggregates, per column: carry[t] = the sums
// carried into tile t.  One workgroup per column: each thread reduces a run of
// consecutive tiles, the thread aggregates are scanned in LDS (Hillis-Steele with the
// segmented operator (f1, s1) + (f2, s2) = (f1 | f2, f2 ? s2 : s1 + s2)), and each thread
// rescans its run with the carry it receives.  The combination order is fixed, so the
// result does not depend on timing.
template <int NT>
__device__ __forceinline__ void carry_scan(const ScanJob &J, const int c)
{
    const int32_t *__restrict__ tileF = J.tileF;
    const double *__restrict__ tileS = J.tileS;
    double *__restrict__ carry = J.carry;
    const int T = (int)J.ntiles, n2 = J.n;
    const int tid = threadIdx.x;
    const int L = (T + NT - 1) / NT;
    const int tb = min(T, tid * L), te = min(T, tb + L);
    __shared__ int sf[2][NT];
    __shared__ double ss[2][NT];
    int F = 0;
    double S = 0.0;
    for (int t = tb; t < te; t++) {
        const int ft = tileF[t];
        const double st = tileS[(int64_t)t * n2 + c];
        S = ft ? st : S + st;
        F |= ft;
    }
    int cur = 0;
    sf[0][tid] = F;
    ss[0][tid] = S;
    __syncthreads();
    for (int off = 1; off < NT; off <<= 1) {
        int f = sf[cur][tid];
        double v = ss[cur][tid];
        if (tid >= off) {
            const int fp = sf[cur][tid - off];
            const double vp = ss[cur][tid - off];
            v = f ? v : vp + v;
            f |= fp;
        }
        sf[cur ^ 1][tid] = f;
        ss[cur ^ 1][tid] = v;
        cur ^= 1;
        __syncthreads();
    }
    double run = tid > 0 ? ss[cur][tid - 1] : 0.0;  // inclusive aggregate of the threads before
    for (int t = tb; t < te; t++) {
        carry[(int64_t)t * n2 + c] = run;
        const int ft = tileF[t];
        const double st = tileS[(int64_t)t * n2 + c];
        run = ft ? st : run + st;
    }
}

// blocks [0, j0.n) take the columns of job 0, the rest those of job 1
__global__ __launch_bounds__(kCarryThreads) void k_carry_scan(ScanJob j0, ScanJob j1)
{
    const bool second = (int)blockIdx.x >= j0.n;
    carry_scan<kCarryThreads>(second ? j1 : j0, (int)blockIdx.x - (second ? j0.n : 0));
}

// A batch (device table): block b scans columns [map[b].y, map[b].y + 64) of job map[b].x.
// Thread (q, c) of the block takes column c of the q-th of 16 chunks of the job's tiles,
// so that a wave reads one tile's aggregates of 64 columns at once (one coalesced read)
// and writes one carry row at once: each chunk's aggregate, then each chunk's carry-in
// from the chunks before it (left to right), then the carries of the chunk's tiles.
constexpr int kCarryChunks = kBatchCarryThreads / 64;
__global__ __launch_bounds__(kBatchCarryThreads) void k_carry_scan_batch(const ScanJob *__restrict__ jobs,
                                                                        const int2 *__restrict__ map)
{
    __shared__ int sf[kCarryChunks][64];
    __shared__ double ss[kCarryChunks][64];
    const int2 e = map[blockIdx.x];
    const ScanJob J = jobs[e.x];
    const int T = (int)J.ntiles, n2 = J.n;
    const int lc = (int)threadIdx.x & 63, q = (int)threadIdx.x >> 6;
    const int c = e.y + lc;
    const bool live = c < n2;
    const int cc = live ? c : n2 - 1;
    const int L = (T + kCarryChunks - 1) / kCarryChunks;
    const int tb = min(T, q * L), te = min(T, tb + L);
    constexpr int U = 8;  // tiles whose aggregates are loaded together
    int F = 0;
    double S = 0.0;
    for (int t0 = tb; t0 < te; t0 += U) {
        int f[U];
        double st[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int t = min(t0 + u, te - 1);
            f[u] = J.tileF[t];
            st[u] = J.tileS[(int64_t)t * n2 + cc];
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            if (t0 + u >= te) break;
            S = f[u] ? st[u] : S + st[u];
            F |= f[u];
        }
    }
    sf[q][lc] = F;
    ss[q][lc] = S;
    __syncthreads();
    double run = 0.0;
    for (int qq = 0; qq < q; qq++) run = sf[qq][lc] ? ss[qq][lc] : run + ss[qq][lc];
    for (int t0 = tb; t0 < te; t0 += U) {
        int f[U];
        double st[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int t = min(t0 + u, te - 1);
            f[u] = J.tileF[t];
            st[u] = J.tileS[(int64_t)t * n2 + cc];
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            if (t0 + u >= te) break;
            if (live) J.carry[(int64_t)(t0 + u) * n2 + c] = run;
            run = f[u] ? st[u] : run + st[u];
        }
    }
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void k_assemble_a(const Tin *__restrict__ A, int64_t lda, int m1,
                                                    int n1, int n2, int tile_rows, Groups g,
                                                    int cartesian, const double *__restrict__ heads,
                                                    Tout *__restrict__ M1)
{
    const int N = n1 + n2;
    const int64_t r0 = (int64_t)blockIdx.x * tile_rows;
    const int G = (int)g.counts[CNT_G];
    __shared__ int s_g0;
    __shared__ int m_g[kMaxTileRows], m_out[kMaxTileRows];
    __shared__ double m_sc[kMaxTileRows];
    if (threadIdx.x == 0) s_g0 = cartesian ? 0 : first_end_gt(g.offA, g.m1, G, r0);
    __syncthreads();
    const int g0 = s_g0;
    for (int r = threadIdx.x; r < tile_rows; r += blockDim.x) {
        const int64_t s = r0 + r;
        int gi = -1;
        if (s < m1 && G > 0) {
            if (cartesian) gi = 0;
            else if (g0 < G) {
                const int cand = last_start_le(g.offA, g0, min(G, g0 + r + 1), s);
                if (g.offA[cand] <= s && s < (int64_t)g.offA[cand] + g.m1[cand]) gi = cand;
            }
        }
        m_g[r] = gi;
        if (gi >= 0) {
            m_out[r] = g.r1[gi] + (int)(s - g.offA[gi]);
            m_sc[r] = sqrt((double)g.m2[gi]);
        }
    }
    __syncthreads();
    const int total = tile_rows * N;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int r = idx / N, col = idx - r * N;
        const int gi = m_g[r];
        if (gi < 0) continue;
        double v;
        if (col < n1) v = m_sc[r] * to_f64(A[(r0 + r) * lda + col]);
        else v = heads[(int64_t)gi * n2 + (col - n1)];
        M1[(int64_t)m_out[r] * N + col] = (Tout)v;
    }
}

__global__ __launch_bounds__(256) void k_head_rows(Groups g, const double *__restrict__ hA,
                                                  const double *__restrict__ hB, int n1, int n2,
                                                  void *out, int out_f64)
{
    const int N = n1 + n2;
    const int64_t G = g.counts[CNT_G];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t gi = e / N;
    const int c = (int)(e - gi * N);
    if (gi >= G) return;
    const double v = c < n1 ? sqrt((double)g.m2[gi]) * hA[gi * n1 + c]
                            : sqrt((double)g.m1[gi]) * hB[gi * n2 + (c - n1)];
    if (out_f64) ((double *)out)[e] = v;
    else ((float *)out)[e] = (float)v;
}

}  // namespace

hipError_t launch_head_rows(Groups g, int64_t gcap, const double *headsA, const double *headsB,
                            int64_t n1, int64_t n2, void *out, int out_f64, hipStream_t s)
{
    const int64_t total = gcap * (n1 + n2);
    if (total == 0) return hipSuccess;
    k_head_rows<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(g, headsA, headsB, (int)n1, (int)n2,
                                                                 out, out_f64);
    return hipGetLastError();
}

ScanPlan scan_plan(int64_t m2, int64_t n2, int in_bytes)
{
    ScanPlan p;
    p.cpt = n2 > kScanThreads ? 2 : 1;
    const int ncolthr = (int)((n2 + p.cpt - 1) / p.cpt);
    p.rpt = 16;
    int q = kScanThreads / (ncolthr > 0 ? ncolthr : 1);
    if (q < 1) q = 1;
    if (q * p.rpt > kMaxTileRows) q = kMaxTileRows / p.rpt;
    p.q = q;
    p.tile_rows = q * p.rpt;
    p.ntiles = (m2 + p.tile_rows - 1) / p.tile_rows;
    (void)in_bytes;
    return p;
}

ScanJob scan_job(const void *X, int64_t ldx, int64_t m, int64_t n, ScanSide side, void *out, double *heads,
                 int32_t *tileF, double *tileS, double *carry, const ScanPlan &sp)
{
    ScanJob j;
    j.in = X;
    j.ld = ldx;
    j.m = (int)m;
    j.n = (int)n;
    j.q = sp.q;
    j.side = side;
    j.out = out;
    j.heads = heads;
    j.tileF = tileF;
    j.tileS = tileS;
    j.carry = carry;
    j.ntiles = sp.ntiles;
    return j;
}

hipError_t launch_seg_scan(const ScanJob &j0_in, const ScanJob &j1_in, int cpt, int in_f64, int out_f64, Groups g,
                           int cartesian, hipStream_t s, int pass)
{
    ScanJob j0 = j0_in, j1 = j1_in;
    j0.g = j1.g = g;
    j0.cartesian = j1.cartesian = cartesian;
    const int64_t tiles = j0.ntiles + j1.ntiles;
    if (tiles == 0) return hipSuccess;
    if (j0.n > kMaxCols || j1.n > kMaxCols) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)tiles;
#define FIGARO_TILE(TI, TO, CPT, WR) \
    k_seg_tile<TI, TO, CPT, 16, WR><<<grid, kScanThreads, 0, s>>>(j0, j1)
#define FIGARO_TILE_ALL(WR)                                                                       \
    do {                                                                                          \
        if (cpt == 1) {                                                                           \
            if (in_f64 && out_f64) FIGARO_TILE(double, double, 1, WR);                            \
            else if (in_f64) FIGARO_TILE(double, float, 1, WR);                                   \
            else if (out_f64) FIGARO_TILE(float, double, 1, WR);                                  \
            else FIGARO_TILE(float, float, 1, WR);                                                \
        } else {                                                                                  \
            if (in_f64 && out_f64) FIGARO_TILE(double, double, 2, WR);                            \
            else if (in_f64) FIGARO_TILE(double, float, 2, WR);                                   \
            else if (out_f64) FIGARO_TILE(float, double, 2, WR);                                  \
            else FIGARO_TILE(float, float, 2, WR);                                                \
        }                                                                                         \
    } while (0)
    hipError_t e;
    if (pass < 0 || pass == 0) {
        FIGARO_TILE_ALL(false);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (pass < 0 || pass == 1) {
        // jobs without tiles have no columns to carry
        ScanJob c0 = j0, c1 = j1;
        if (c0.ntiles == 0) c0.n = 0;
        if (c1.ntiles == 0) c1.n = 0;
        k_carry_scan<<<(unsigned)(c0.n + c1.n), kCarryThreads, 0, s>>>(c0, c1);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (pass < 0 || pass == 2) FIGARO_TILE_ALL(true);
#undef FIGARO_TILE_ALL
#undef FIGARO_TILE
    return hipGetLastError();
}

hipError_t launch_seg_scan_batch(int pass, const ScanJob *jobs, const int2 *tile_map, int64_t ntiles,
                                 const int2 *col_map, int64_t ncols, int cpt, int in_f64, int out_f64, hipStream_t s)
{
    if (ntiles == 0) return hipSuccess;
    if (ntiles > INT32_MAX || ncols > INT32_MAX) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)ntiles;
#define FIGARO_TILE(TI, TO, CPT, WR) \
    k_seg_tile_batch<TI, TO, CPT, 16, WR><<<grid, kScanThreads, 0, s>>>(jobs, tile_map)
#define FIGARO_TILE_ALL(WR)                                                                       \
    do {                                                                                          \
        if (cpt == 1) {                                                                           \
            if (in_f64 && out_f64) FIGARO_TILE(double, double, 1, WR);                            \
            else if (in_f64) FIGARO_TILE(double, float, 1, WR);                                   \
            else if (out_f64) FIGARO_TILE(float, double, 1, WR);                                  \
            else FIGARO_TILE(float, float, 1, WR);                                                \
        } else {                                                                                  \
            if (in_f64 && out_f64) FIGARO_TILE(double, double, 2, WR);                            \
            else if (in_f64) FIGARO_TILE(double, float, 2, WR);                                   \
            else if (out_f64) FIGARO_TILE(float, double, 2, WR);                                  \
            else FIGARO_TILE(float, float, 2, WR);                                                \
        }                                                                                         \
    } while (0)
    if (pass == 0) FIGARO_TILE_ALL(false);
    else if (pass == 1) {
        if (ncols > 0) k_carry_scan_batch<<<(unsigned)ncols, kBatchCarryThreads, 0, s>>>(jobs, col_map);
    } else {
        FIGARO_TILE_ALL(true);
    }
#undef FIGARO_TILE_ALL
#undef FIGARO_TILE
    return hipGetLastError();
}

hipError_t launch_assemble_a(const void *A, int in_f64, int64_t lda, int64_t m1, int64_t n1,
                             int64_t n2, Groups g, int cartesian, const double *heads, void *M1,
                             int out_f64, hipStream_t s)
{
    if (m1 == 0) return hipSuccess;
    const int N = (int)(n1 + n2);
    int tile_rows = 4096 / N;
    if (tile_rows < 1) tile_rows = 1;
    if (tile_rows > kMaxTileRows) tile_rows = kMaxTileRows;
    const unsigned grid = (unsigned)((m1 + tile_rows - 1) / tile_rows);
#define FIGARO_ASM(TI, TO)                                                                         \
    k_assemble_a<TI, TO><<<grid, 256, 0, s>>>((const TI *)A, lda, (int)m1, (int)n1, (int)n2,      \
                                              tile_rows, g, cartesian, heads, (TO *)M1)
    if (in_f64 && out_f64) FIGARO_ASM(double, double);
    else if (in_f64) FIGARO_ASM(double, float);
    else if (out_f64) FIGARO_ASM(float, double);
    else FIGARO_ASM(float, float);
#undef FIGARO_ASM
    return hipGetLastError();
}

}  // namespace figaro
