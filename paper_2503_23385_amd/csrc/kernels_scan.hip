// Per-group QR head and tail of B, and assembly of region 1 of the compact
// matrix ("Figaro on GPUs: Two Tables", Section 1: the head operator
// H(B) = (1/sqrt m) sum_i B_i, the tail operator
// T(B)_i = (sqrt(i) B_{i+1} - S_i / sqrt(i)) / sqrt(i+1) with S_i the sum of the
// first i rows, and Claim 1's compact form).
//
// Head/tail: one pass over B.  Rows are cut into tiles; a tile is taken by a
// workgroup in ticket order, each thread owns one column (or two) of a
// contiguous run of rows, keeps the rows in registers and accumulates FP64
// running sums that restart at every group start.  Carries across tiles come
// from a decoupled look-back over per-tile aggregates, so B is read from HBM
// exactly once.  A tail row i of group g goes to region-2 row r2_g + i - 1,
// scaled by sqrt(m1_g); the head goes to heads[g] (FP64).
//
// Region 1: row r of A in group g becomes [sqrt(m2_g) A_r | H(B_g)] at row
// r1_g + (r - offA_g).
#include "common.h"

namespace figaro {
namespace {

constexpr int kScanThreads = 256;
constexpr int kMaxTileRows = 512;
constexpr int kMaxCols = 512;
constexpr int kLookbackSpinLimit = 1 << 24;

constexpr int FLAG_EMPTY = 0, FLAG_AGG = 1, FLAG_INCL = 2;

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

template <typename Tin, typename Tout, int CPT, int RPT>
__global__ __launch_bounds__(kScanThreads) void k_seg_scan(
    const Tin *__restrict__ B, int64_t ldb, int m2, int n2, int Q, Groups g, int cartesian,
    Tout *__restrict__ M2, double *__restrict__ heads, int32_t *flags, double *agg, double *incl,
    int32_t *ticket, int32_t *status, int ntiles)
{
    const int tid = threadIdx.x;
    const int ncolthr = (n2 + CPT - 1) / CPT;
    const int c = tid % ncolthr;
    const int q = tid / ncolthr;
    const bool active = q < Q;
    const int TR = Q * RPT;

    __shared__ int s_tile, s_g0, s_need;
    __shared__ int m_g[kMaxTileRows], m_pos[kMaxTileRows], m_out[kMaxTileRows];
    __shared__ double m_c1[kMaxTileRows], m_c2[kMaxTileRows], m_hs[kMaxTileRows];
    __shared__ int a_f[kScanThreads];
    __shared__ double a_s[kMaxCols];
    __shared__ double carry[kMaxCols];

    if (tid == 0) s_tile = atomicAdd(ticket, 1);
    __syncthreads();
    const int t = s_tile;
    if (t >= ntiles) return;  // uniform
    const int64_t t0 = (int64_t)t * TR;
    const int G = (int)g.counts[CNT_G];

    // Issue the tile's loads first; they stay in flight during the row metadata search.
    double x[RPT][CPT];
#pragma unroll
    for (int i = 0; i < RPT; i++) {
        const int64_t s = t0 + (int64_t)q * RPT + i;
#pragma unroll
        for (int cc = 0; cc < CPT; cc++) {
            const int col = c + cc * ncolthr;
            x[i][cc] = (active && s < m2 && col < n2) ? to_f64(B[s * ldb + col]) : 0.0;
        }
    }

    if (tid == 0) s_g0 = cartesian ? 0 : first_end_gt(g.offB, g.m2, G, t0);
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
                const int cand = last_start_le(g.offB, g0, hi, s);
                if (g.offB[cand] <= s && s < (int64_t)g.offB[cand] + g.m2[cand]) {
                    gi = cand;
                    pos = (int)(s - g.offB[cand]);
                }
            }
        }
        m_g[r] = gi;
        m_pos[r] = pos;
        if (gi >= 0) {
            const double sm1 = sqrt((double)g.m1[gi]);
            const int m2g = g.m2[gi];
            m_out[r] = g.r2[gi] + pos - 1;
            if (pos > 0) {
                const double sp = sqrt((double)pos), sp1 = sqrt((double)pos + 1.0);
                m_c1[r] = sm1 * sp / sp1;
                m_c2[r] = sm1 / (sp * sp1);
            }
            m_hs[r] = (pos == m2g - 1) ? 1.0 / sqrt((double)m2g) : 0.0;
        }
    }
    __syncthreads();

    // Thread aggregate over its rows: (f, s) with f = "a segment starts here".
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
    }
    // Row-group aggregates to LDS: a_f[q], a_s[q * n2 + col].
    if (active && c == 0) a_f[q] = f;
    if (active) {
#pragma unroll
        for (int cc = 0; cc < CPT; cc++) {
            const int col = c + cc * ncolthr;
            if (col < n2) a_s[q * n2 + col] = sacc[cc];
        }
    }
    if (tid == 0) s_need = (m_g[0] >= 0 && m_pos[0] > 0) ? 1 : 0;
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
    // Every thread computed the same F (it depends on rows only); thread 0's copy is used.
    __shared__ int s_F;
    if (tid == 0) s_F = F;
    __syncthreads();
    const int tileF = s_F;
    const int need = s_need;

    // Publish this tile's aggregate (or its inclusive prefix when it holds a segment start).
    if (active && q == 0) {
#pragma unroll
        for (int cc = 0; cc < CPT; cc++) {
            const int col = c + cc * ncolthr;
            if (col < n2) {
                if (tileF || t == 0) incl[(int64_t)t * n2 + col] = S[cc];
                else agg[(int64_t)t * n2 + col] = S[cc];
            }
        }
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(&flags[t], (tileF || t == 0) ? FLAG_INCL : FLAG_AGG, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }

    // Decoupled look-back for the carry into the tile's first (continuing) group.
    if (need && tid < 64) {
        double acc[kMaxCols / 64];
#pragma unroll
        for (int k = 0; k < kMaxCols / 64; k++) acc[k] = 0.0;
        int j = t - 1;
        int spins = 0;
        bool timed_out = false;
        while (j >= 0) {
            int fl = __hip_atomic_load(&flags[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            while (fl == FLAG_EMPTY) {
                if (++spins > kLookbackSpinLimit) { timed_out = true; break; }
                __builtin_amdgcn_s_sleep(2);
                fl = __hip_atomic_load(&flags[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (timed_out) break;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const double *src = (fl == FLAG_INCL) ? incl : agg;
#pragma unroll
            for (int k = 0; k < kMaxCols / 64; k++) {
                const int col = tid + 64 * k;
                if (col < n2)
                    acc[k] += __hip_atomic_load(&src[(int64_t)j * n2 + col], __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
            }
            if (fl == FLAG_INCL) break;
            j--;
        }
        if (timed_out && tid == 0) atomicExch(status, kStatusTimeout);
#pragma unroll
        for (int k = 0; k < kMaxCols / 64; k++) {
            const int col = tid + 64 * k;
            if (col < n2) carry[col] = acc[k];
        }
    }
    __syncthreads();

    if (need && !tileF) {
        // Inclusive prefix for successors: carry + this tile's sum.
        if (active && q == 0) {
#pragma unroll
            for (int cc = 0; cc < CPT; cc++) {
                const int col = c + cc * ncolthr;
                if (col < n2) incl[(int64_t)t * n2 + col] = carry[col] + S[cc];
            }
        }
        __threadfence();
        __syncthreads();
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_store(&flags[t], FLAG_INCL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }

    // Second pass: tails and heads with the running FP64 prefix.
    if (!active) return;
    double run[CPT];
#pragma unroll
    for (int cc = 0; cc < CPT; cc++) {
        const int col = c + cc * ncolthr;
        const double cin = (need && col < n2) ? carry[col] : 0.0;
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

}  // namespace

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

hipError_t launch_seg_scan(const void *B, int in_f64, int64_t ldb, int64_t m2, int64_t n2,
                           Groups g, int cartesian, void *M2, int out_f64, double *heads,
                           int32_t *flags, double *agg, double *incl, int32_t *ticket,
                           int32_t *status, const ScanPlan &sp, hipStream_t s)
{
    if (sp.ntiles == 0) return hipSuccess;
    if (n2 > kMaxCols) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)sp.ntiles;
#define FIGARO_SCAN(TI, TO, CPT)                                                                  \
    k_seg_scan<TI, TO, CPT, 16><<<grid, kScanThreads, 0, s>>>(                                   \
        (const TI *)B, ldb, (int)m2, (int)n2, sp.q, g, cartesian, (TO *)M2, heads, flags, agg,    \
        incl, ticket, status, (int)sp.ntiles)
    if (sp.cpt == 1) {
        if (in_f64 && out_f64) FIGARO_SCAN(double, double, 1);
        else if (in_f64) FIGARO_SCAN(double, float, 1);
        else if (out_f64) FIGARO_SCAN(float, double, 1);
        else FIGARO_SCAN(float, float, 1);
    } else {
        if (in_f64 && out_f64) FIGARO_SCAN(double, double, 2);
        else if (in_f64) FIGARO_SCAN(double, float, 2);
        else if (out_f64) FIGARO_SCAN(float, double, 2);
        else FIGARO_SCAN(float, float, 2);
    }
#undef FIGARO_SCAN
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
