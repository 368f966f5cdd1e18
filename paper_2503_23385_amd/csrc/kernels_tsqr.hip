// Householder TSQR of the compact matrix (the QR step of the paper's
// pipeline, Experiments section: a dense Householder QR of the concatenated
// heads and tails; here a tall-skinny reduction instead of a library geqrf).
//
// The unit of work is one upper triangle R that absorbs blocks X of rows:
//     R <- triu(QR([R; X])).
// Reflector j involves only row j of R and column j of X (structured TSQR).
// With alpha = R_jj, d_k = x_j . x_k (so d_j = |x_j|^2) and
//     beta = -sign(alpha) sqrt(alpha^2 + d_j),  tau = 1 - alpha / beta,
// the reflector with v = x_j / (alpha - beta) updates, for k > j,
//     w_k = R_jk + d_k / (alpha - beta),  R_jk -= tau w_k,  x_k += (w_k / beta) x_j,
// and sets R_jj = beta (tau * scale = -1 / beta folded in).  Q is never formed.
//
// Widths up to 64: one wave owns one triangle (packed in LDS) and keeps a block
// of X in registers -- at padded widths 16 to 64 lane 16 g + p holds columns
// p, p + 16, ... of row group g and column j reaches each group by a lane
// permutation; at widths 4 and 8 lane (k, h) holds column k of row set h and
// column j is broadcast through a per-wave LDS slot.  Every reduction stays
// inside the wave -- no workgroup barrier.  A region is reduced in one launch: each wave
// reduces its rows to a leaf triangle, then the waves climb a tree whose arity
// is set so that one block of rows holds all siblings of a node; at each node
// the last child to arrive (per-node atomic counter) combines them, always as
// the first child absorbing the others in child order, so results do not
// depend on timing; the others exit.  Nothing waits on anything.
//
// Wider rows (padded widths 128 to 512) go to the blocked panel kernel
// (kernels_panel.hip); its tree levels are separate launches.
#include <float.h>

#include <type_traits>

#include "common.h"

namespace figaro {
namespace {

constexpr int kWavesPerBlock = 4;

__host__ __device__ constexpr int packed_size(int np) { return np * (np + 1) / 2; }
__device__ inline int pidx(int np, int j, int k) { return j * np - (j * (j - 1)) / 2 + (k - j); }

template <typename T>
__device__ inline T shfl_xor_t(T v, int m) { return __shfl_xor(v, m, 64); }

template <typename Tin, typename Tacc>
__device__ inline Tacc load_src(const RowSrc &s, int64_t lr, int k)
{
    const int c = k - s.col_off;
    if (c < 0 || c >= s.width) return Tacc(0);
    return (Tacc)((const Tin *)s.p)[lr * s.ld + c];
}

__device__ inline int64_t src_rows(const RowSrc &s) { return s.rows_dev ? *s.rows_dev : s.rows_host; }

__device__ inline double readlane_f64(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

__device__ inline double readlane_t(double v, int l) { return readlane_f64(v, l); }
__device__ inline float readlane_t(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Hardware reciprocal / reciprocal square root refined by two Newton steps.
__device__ inline double rcp_refined(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    r = fma(fma(-x, r, 1.0), r, r);
    return r;
}
__device__ inline double rsq_refined(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * fma(-hx * y, y, 1.5);
    y = y * fma(-hx * y, y, 1.5);
    return y;
}

// ------------------------------------------------------------------ one wave per triangle (NP <= 64)

template <int NP>
struct WaveGeom {
    static constexpr int H = NP >= 64 ? 1 : 64 / NP;    // row sets per wave
    static constexpr int RPT = 32;                      // rows per lane per block
    static constexpr int BR = H * RPT;                  // rows per block
    static constexpr int PS = packed_size(NP);
};

__host__ __device__ constexpr int wave_block_rows(int np) { return (np >= 64 ? 1 : 64 / np) * 32; }

// Absorb one block (RPT rows per lane, already in x) into R for columns [jstart, width).
template <int NP, typename Tacc>
__device__ inline void wave_block(Tacc (&x)[WaveGeom<NP>::RPT], Tacc *Rp, Tacc *xb, int k, int h,
                                  int jstart, int width)
{
    constexpr int RPT = WaveGeom<NP>::RPT;
    const bool col_ok = k < width;
    for (int j = jstart; j < width; j++) {
        __builtin_amdgcn_wave_barrier();
        if (k == j) {
#pragma unroll
            for (int i = 0; i < RPT; i++) xb[i] = x[i];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        Tacc xj[RPT];
#pragma unroll
        for (int i = 0; i < RPT; i++) xj[i] = xb[i];
        const double alpha = (double)Rp[pidx(NP, j, j)];
        const Tacc rjk = (k > j && col_ok) ? Rp[pidx(NP, j, k)] : Tacc(0);
        Tacc dp[4] = {Tacc(0), Tacc(0), Tacc(0), Tacc(0)};
#pragma unroll
        for (int i = 0; i < RPT; i++) dp[i & 3] += xj[i] * x[i];
        Tacc d = (dp[0] + dp[1]) + (dp[2] + dp[3]);
#pragma unroll
        for (int off = NP; off < 64; off <<= 1) d += shfl_xor_t(d, off);
        double s;
        if constexpr (sizeof(Tacc) == 8) {
            s = readlane_f64(d, j);
        } else {
            // reflector scalars in FP64 for the FP32 form
            double sp[2] = {0.0, 0.0};
#pragma unroll
            for (int i = 0; i < RPT; i++) sp[i & 1] += (double)xj[i] * (double)xj[i];
            double sd = sp[0] + sp[1];
#pragma unroll
            for (int off = NP; off < 64; off <<= 1) sd += shfl_xor_t(sd, off);
            s = readlane_f64(sd, j);
        }
        const double q = fma(alpha, alpha, s);
        // A column whose norm is below the normal range is left untouched (tau = 0).
        if (s > 0.0 && q >= DBL_MIN) {
            const double r = rsq_refined(q);  // 1 / |(alpha, x_j)|
            const double sg = alpha >= 0.0 ? 1.0 : -1.0;
            const double nrm = q * r;
            const double beta = -sg * nrm;
            const double inv_beta = -sg * r;
            const double scl = rcp_refined(alpha + sg * nrm);  // 1 / (alpha - beta)
            const double tau = 1.0 - alpha * inv_beta;
            if (k > j && col_ok) {
                const double w = (double)rjk + scl * (double)d;
                if (h == 0) Rp[pidx(NP, j, k)] = (Tacc)((double)rjk - tau * w);
                const Tacc c = (Tacc)(w * inv_beta);
#pragma unroll
                for (int i = 0; i < RPT; i++) x[i] += c * xj[i];
            }
            if (k == j && h == 0) Rp[pidx(NP, j, j)] = (Tacc)beta;
        }
    }
}

// R <- triangle T (width rows of ld doubles, entries left of the diagonal ignored).
template <int NP, typename Tacc>
__device__ inline void wave_init_tri(Tacc *Rp, const double *T, int64_t ld, int width, int lane)
{
    staged_copy<16, double>(
        width * NP, lane, 64,
        [&](int e) {
            const int j = e / NP, kk = e - j * NP;
            return T[(int64_t)j * ld + (kk < width ? kk : width - 1)];
        },
        [&](int e, double v) {
            const int j = e / NP, kk = e - j * NP;
            if (kk >= j) Rp[pidx(NP, j, kk)] = kk < width ? (Tacc)v : Tacc(0);
        });
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <int NP, typename Tacc>
__device__ inline void wave_zero(Tacc *Rp, int lane)
{
    for (int e = lane; e < WaveGeom<NP>::PS; e += 64) Rp[e] = Tacc(0);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <int NP, typename Tacc>
__device__ inline void wave_store(const Tacc *Rp, double *out, int width, int lane)
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int e = lane; e < width * NP; e += 64) {
        const int j = e / NP, kk = e - j * NP;
        out[e] = (kk >= j && kk < width) ? (double)Rp[pidx(NP, j, kk)] : 0.0;
    }
}

// Absorb a triangle of `trows` rows (ld doubles each) whose columns sit at [off, off + tw):
// row i has nonzeros only from column off + i on.
template <int NP, typename Tacc>
__device__ inline void wave_absorb_tri(Tacc *Rp, Tacc *xb, const double *T, int64_t ld, int trows,
                                       int off, int tw, int width, int k, int h)
{
    constexpr int RPT = WaveGeom<NP>::RPT, BR = WaveGeom<NP>::BR;
    const int c = k - off, cc = c < 0 ? 0 : (c < tw ? c : tw - 1);
    for (int b0 = 0; b0 < trows; b0 += BR) {
        // unconditional loads (row and column clamped into T), masked afterwards
        Tacc x[RPT];
#pragma unroll
        for (int i = 0; i < RPT; i++) {
            const int r = b0 + h * RPT + i;
            x[i] = (Tacc)T[(int64_t)(r < trows ? r : trows - 1) * ld + cc];
        }
#pragma unroll
        for (int i = 0; i < RPT; i++) {
            const int r = b0 + h * RPT + i;
            if (!(r < trows && c >= 0 && c < tw)) x[i] = Tacc(0);
        }
        wave_block<NP, Tacc>(x, Rp, xb, k, h, off + b0, width);
    }
}

// Absorb rows [r0, r1) of up to two sources (concatenated) in blocks.
template <int NP, typename Tin, typename Tacc>
__device__ inline void wave_absorb_rows(Tacc *Rp, Tacc *xb, const RowSrc &s0, const RowSrc &s1,
                                        int64_t rows0, int64_t r0, int64_t r1, int tri_rows,
                                        int width, int k, int h)
{
    constexpr int RPT = WaveGeom<NP>::RPT, BR = WaveGeom<NP>::BR;
    for (int64_t rb = r0; rb < r1; rb += BR) {
        // unconditional loads (clamped into the sources), masked afterwards
        Tacc x[RPT];
#pragma unroll
        for (int i = 0; i < RPT; i++) {
            const int64_t r = rb + h * RPT + i;
            x[i] = load_stacked<Tin, Tacc>(s0, s1, rows0, r < r1 ? r : r1 - 1, k);
        }
#pragma unroll
        for (int i = 0; i < RPT; i++) {
            const int64_t r = rb + h * RPT + i;
            if (!(r < r1 && k < width && stacked_real(s0, s1, rows0, r, k))) x[i] = Tacc(0);
        }
        int jstart = 0;
        const int64_t rlast = min(r1, rb + BR) - 1;
        if (rlast < rows0) jstart = s0.col_off;
        else if (rb >= rows0) jstart = s1.col_off;
        if (tri_rows > 0 && (rlast < rows0 || rb >= rows0)) {
            const int64_t lr = rb < rows0 ? rb : rb - rows0;
            const int64_t off = lr % tri_rows;
            if (off + BR <= tri_rows) jstart += (int)off;
        }
        wave_block<NP, Tacc>(x, Rp, xb, k, h, jstart, width);
    }
}

// Rows of s0 then s1 reduced into ntri triangles (optionally starting from `init`).
template <int NP, typename Tin, typename Tacc>
__global__ __launch_bounds__(64 * kWavesPerBlock) void k_tsqr_wave(const double *init, int64_t init_ld,
                                                                  RowSrc s0, RowSrc s1, int nsrc,
                                                                  int width, int tri_rows, int ntri,
                                                                  double *tri_out, int64_t tri_stride)
{
    using Gm = WaveGeom<NP>;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int gw = blockIdx.x * kWavesPerBlock + wv;
    const int k = lane % NP, h = lane / NP;
    __shared__ Tacc Rs[kWavesPerBlock][Gm::PS];
    __shared__ __align__(16) Tacc Xs[kWavesPerBlock][Gm::BR];
    if (gw >= ntri) return;  // waves are independent: no block-level barrier follows
    Tacc *Rp = Rs[wv];
    Tacc *xb = Xs[wv] + h * Gm::RPT;
    if (init) wave_init_tri<NP, Tacc>(Rp, init, init_ld, width, lane);
    else wave_zero<NP, Tacc>(Rp, lane);
    const int64_t rows0 = src_rows(s0);
    const int64_t total = rows0 + (nsrc > 1 ? src_rows(s1) : 0);
    int64_t chunk = (total + ntri - 1) / ntri;
    chunk = ((chunk + Gm::BR - 1) / Gm::BR) * Gm::BR;
    const int64_t r0 = (int64_t)gw * chunk, r1 = min(total, r0 + chunk);
    wave_absorb_rows<NP, Tin, Tacc>(Rp, xb, s0, s1, rows0, r0, r1, tri_rows, width, k, h);
    wave_store<NP, Tacc>(Rp, tri_out + (int64_t)gw * tri_stride, width, lane);
}

// ------------------------------------------------------------------ one workgroup per triangle (tree)
//
// The waves of a workgroup share one triangle R and each holds its share of the
// current block (BR rows per wave).  Column step j: every wave forms its partial dot
// products d_k over its own rows, the partials meet in LDS (one barrier; summed in a
// fixed order, so the result does not depend on timing), every wave computes the same
// reflector scalars and updates its own rows.  Only step j changes row j of R; every wave reads it at the start of the
// step, before the barrier, and its new values are written one step later, after the
// next barrier.

// Waves per workgroup of the tree kernel (measured): 8 at padded width 32, where the
// blocks of 512 rows halve the sequential column steps of a leaf and two waves per SIMD
// hide part of the LDS broadcast; 4 elsewhere (8 measured slower at widths 64 and below 32).
__host__ __device__ constexpr int tree_waves(int np) { return np == 32 ? 8 : 4; }

// Sum of the values of lanes l and l ^ 32, the same in both lanes: a swap of the wave's
// halves (a VALU lane permutation, no LDS round trip) and one add.
__device__ inline double half_swap_sum(double v)
{
    const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
    const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}

// Row stride (doubles) of the partial-sum table, one row per column with the waves'
// partials side by side: a lane reads its column's partials with 128-bit reads; the two
// extra doubles spread the rows over the LDS banks.
__host__ __device__ constexpr int tree_red_stride(int np) { return tree_waves(np) + 2; }

template <int NP, typename Tacc>
struct WgState {
    Tacc *R;             // packed triangle (LDS)
    Tacc *xb;            // this wave's broadcast slot, offset by the row set h
    double (*red)[NP][tree_red_stride(NP)];  // [parity][column][wave]
    int k, h, wv, par;
    int pend_row;        // row of R whose new values are still in pend_val (-1: none)
    Tacc pend_val;
};

template <int NP, typename Tacc>
__device__ inline void wg_flush(WgState<NP, Tacc> &st, int width)
{
    if (st.pend_row >= 0 && st.wv == 0 && st.h == 0 && st.k >= st.pend_row && st.k < width)
        st.R[pidx(NP, st.pend_row, st.k)] = st.pend_val;
    st.pend_row = -1;
}

// Absorb one block (this wave's RPT rows per lane in x) for columns [jstart, width).
template <int NP, typename Tacc>
__device__ inline void wg_block(Tacc (&x)[WaveGeom<NP>::RPT], WgState<NP, Tacc> &st, int jstart, int width)
{
    constexpr int RPT = WaveGeom<NP>::RPT, H = WaveGeom<NP>::H;
    constexpr int NPART = tree_waves(NP);
    const int k = st.k;
    const bool col_ok = k < width;
    for (int j = jstart; j < width; j++) {
        // Row j of R (changed by this step only), read before the barrier.
        const double alpha = (double)st.R[pidx(NP, j, j)];
        const Tacc rjk = st.R[pidx(NP, j, (k > j && col_ok) ? k : j)];
        // Column j of this wave's rows.  With one row set per wave it is read from lane j
        // into scalar registers (no LDS traffic); with several, lane j of each row set
        // stages it in LDS (a per-row-set select of lane reads costs more than that).
        Tacc xj[RPT];
        if constexpr (H == 1) {
#pragma unroll
            for (int i = 0; i < RPT; i++) xj[i] = readlane_t(x[i], j);
        } else {
            __builtin_amdgcn_wave_barrier();
            if (k == j) {
#pragma unroll
                for (int i = 0; i < RPT; i++) st.xb[i] = x[i];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int i = 0; i < RPT; i++) xj[i] = st.xb[i];
        }
        // Per-lane dot over RPT rows in the accumulation type (FP32 storage: FP32 sums of
        // RPT products, in 8 chains of RPT / 8 fmas), then FP64 from the half-wave sums on.
        Tacc dp[8];
#pragma unroll
        for (int i = 0; i < 8; i++) dp[i] = xj[i] * x[i];
#pragma unroll
        for (int i = 8; i < RPT; i++) dp[i & 7] = fma(xj[i], x[i], dp[i & 7]);
        double d = (double)(((dp[0] + dp[1]) + (dp[2] + dp[3])) + ((dp[4] + dp[5]) + (dp[6] + dp[7])));
#pragma unroll
        for (int off = NP; off < 32; off <<= 1) d += __shfl_xor(d, off, 64);
        if constexpr (H >= 2) d = half_swap_sum(d);
        if (st.h == 0) st.red[st.par][k][st.wv] = d;
        __syncthreads();
        wg_flush(st, width);
        // this lane's column sum; the pivot column's (the same sum, formed the same way by
        // lane j) comes by a lane read instead of another round of LDS reads
        double pk[NPART];
#pragma unroll
        for (int w = 0; w < NPART; w++) pk[w] = st.red[st.par][k][w];
#pragma unroll
        for (int w = 1; w < NPART; w <<= 1)
#pragma unroll
            for (int u = 0; u + w < NPART; u += 2 * w) pk[u] += pk[u + w];
        const double dk = pk[0], s = readlane_f64(dk, j);
        st.par ^= 1;
        const double q = fma(alpha, alpha, s);
        // A column whose norm is below the normal range is left untouched (tau = 0).  The
        // scalars are formed without a branch (the same in every lane), so that the
        // partials of both columns are read together right after the barrier.
        const bool ok = s > 0.0 && q >= DBL_MIN;
        const double r = rsq_refined(ok ? q : 1.0);
        const double sg = alpha >= 0.0 ? 1.0 : -1.0;
        const double nrm = q * r;
        const double beta = -sg * nrm;
        const double inv_beta = -sg * r;
        const double scl = rcp_refined(ok ? alpha + sg * nrm : 1.0);
        const double tau = 1.0 - alpha * inv_beta;
        const double w = (double)rjk + scl * dk;
        const bool upd = ok && k > j && col_ok;
        const Tacc c = upd ? (Tacc)(w * inv_beta) : Tacc(0);
        if (upd) {
#pragma unroll
            for (int i = 0; i < RPT; i++) x[i] += c * xj[i];
        }
        if (ok) {
            st.pend_val = upd ? (Tacc)((double)rjk - tau * w) : (k == j ? (Tacc)beta : Tacc(0));
            st.pend_row = j;
        }
    }
}

// Absorb rows [r0, r1) of src in blocks of WV BR rows (wave wv takes the wv-th share).
// STAGED: every row load is issued unconditionally (row clamped into the source: the
// row pointer advances while the next row is still inside) and masked afterwards, so
// the loads of a block stay in flight together; more registers, used when a launch has
// at most one leaf per compute unit (each leaf's latency is the launch's).  With FP32
// storage the next block's loads are also issued before the current block's column
// steps, which hide them.  Otherwise the loads are conditional (fewer registers, more
// workgroups per compute unit to hide latency with).
template <int NP, typename Tin, typename Tacc, bool STAGED>
__device__ inline void wg_absorb_rows(WgState<NP, Tacc> &st, const RowSrc &src, int64_t r0, int64_t r1,
                                      int tri_rows, int width)
{
    constexpr int RPT = WaveGeom<NP>::RPT, BR = WaveGeom<NP>::BR, BG = tree_waves(NP) * BR;
    constexpr bool PREFETCH = STAGED && sizeof(Tin) == 4 && sizeof(Tacc) == 4;
    // this lane's column of the source, clamped into range (col_in: whether it is real)
    const int c = st.k - src.col_off;
    const bool col_in = st.k < width && c >= 0 && c < src.width;
    const Tin *col_base = (const Tin *)src.p + (c < 0 ? 0 : (c < src.width ? c : src.width - 1));
    const int64_t roff = (int64_t)st.wv * BR + st.h * RPT;  // this lane's first row in a block
    auto load_rows = [&](Tacc (&y)[RPT], int64_t rb) {
        const int64_t rs = rb + roff, last = r1 - 1;
        const Tin *p = col_base + (rs < last ? rs : last) * src.ld;
#pragma unroll
        for (int i = 0; i < RPT; i++) {
            y[i] = (Tacc)*p;
            if (rs + i < last) p += src.ld;
        }
    };
    auto mask_rows = [&](Tacc (&y)[RPT], int64_t rb) {
#pragma unroll
        for (int i = 0; i < RPT; i++)
            if (!(rb + roff + i < r1 && col_in)) y[i] = Tacc(0);
    };
    Tacc xn[PREFETCH ? RPT : 1];
    if constexpr (PREFETCH) {
        if (r0 < r1) load_rows(xn, r0);
    }
    for (int64_t rb = r0; rb < r1; rb += BG) {
        if (st.pend_row >= 0) {  // the block may start at the pending row: write it first
            __syncthreads();
            wg_flush(st, width);
            __syncthreads();
        }
        Tacc x[RPT];
        if constexpr (PREFETCH) {
#pragma unroll
            for (int i = 0; i < RPT; i++) x[i] = xn[i];
            mask_rows(x, rb);
            if (rb + BG < r1) load_rows(xn, rb + BG);
        } else if constexpr (STAGED) {
            load_rows(x, rb);
            mask_rows(x, rb);
        } else {
#pragma unroll
            for (int i = 0; i < RPT; i++) {
                const int64_t r = rb + roff + i;
                x[i] = (r < r1 && col_in) ? (Tacc)col_base[r * src.ld] : Tacc(0);
            }
        }
        int jstart = src.col_off;
        if (tri_rows > 0) {
            const int64_t off = rb % tri_rows;
            if (off + BG <= tri_rows) jstart += (int)off;
        }
        wg_block<NP, Tacc>(x, st, jstart, width);
    }
}

template <int NP, typename Tacc>
__device__ inline void wg_store(WgState<NP, Tacc> &st, double *out, int width)
{
    __syncthreads();
    wg_flush(st, width);
    __syncthreads();
    for (int e = threadIdx.x; e < width * NP; e += 64 * tree_waves(NP)) {
        const int j = e / NP, kk = e - j * NP;
        out[e] = (kk >= j && kk < width) ? (double)st.R[pidx(NP, j, kk)] : 0.0;
    }
}

template <int NP, typename Tacc>
__device__ inline void wg_load_tri(WgState<NP, Tacc> &st, const double *T, int width)
{
    for (int e = threadIdx.x; e < WaveGeom<NP>::PS; e += 64 * tree_waves(NP)) st.R[e] = Tacc(0);
    __syncthreads();
    if (T) {
        staged_copy<8, double>(
            width * NP, threadIdx.x, 64 * tree_waves(NP), [&](int e) { return T[e]; },
            [&](int e, double v) {
                const int j = e / NP, kk = e - j * NP;
                if (kk >= j && kk < width) st.R[pidx(NP, j, kk)] = (Tacc)v;
            });
    }
    __syncthreads();
}

// Up to two regions (same width class) in one launch: workgroups [0, leaves0) reduce
// region 0, the rest region 1.  Each region: one leaf triangle per workgroup, then a
// tree of the region's arity; at each node the last child to arrive (per-node atomic
// counter) combines all children in child order.  slots: the node triangles of every
// level (width x NP doubles each); counters: one int per parent node, zero on entry.
// Leaf g of region rg, then the climb of its tree.
template <int NP, typename Tin, typename Tacc, bool STAGED>
__device__ __forceinline__ void tree_leaf(const TreeRegion &rg, const int g)
{
    using Gm = WaveGeom<NP>;
    constexpr int WV = tree_waves(NP);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    __shared__ Tacc Rs[Gm::PS];
    __shared__ __align__(16) Tacc Xs[WV][Gm::BR];
    __shared__ __align__(16) double red[2][NP][tree_red_stride(NP)];
    __shared__ int s_old;
    const int width = rg.width;
    const int64_t rows = src_rows(rg.src);
    // leaves follow the device-side row count; surplus workgroups leave at once
    const int64_t want = (rows + rg.rows_per_leaf - 1) / rg.rows_per_leaf;
    const int nleaves = (int)max((int64_t)1, min((int64_t)rg.nleaves, want));
    if (g >= nleaves) return;
    WgState<NP, Tacc> st;
    st.R = Rs;
    st.k = lane % NP;
    st.h = lane / NP;
    st.wv = wv;
    st.xb = Xs[wv] + st.h * Gm::RPT;
    st.red = red;
    st.par = 0;
    st.pend_row = -1;
    st.pend_val = Tacc(0);
    wg_load_tri<NP, Tacc>(st, nullptr, width);
    constexpr int BG = WV * Gm::BR;
    int64_t chunk = (rows + nleaves - 1) / nleaves;
    chunk = ((chunk + BG - 1) / BG) * BG;
    const int64_t r0 = (int64_t)g * chunk, r1 = min(rows, r0 + chunk);
    wg_absorb_rows<NP, Tin, Tacc, STAGED>(st, rg.src, r0, r1, 0, width);

    const int64_t tsz = (int64_t)width * NP;
    const int A = rg.arity;
    int node = g, n = nleaves;
    int64_t soff = 0, coff = 0;
    while (n > 1) {
        const int parent = node / A, first = parent * A;
        const int nchild = min(A, n - first);
        if (nchild > 1) {
            wg_store<NP, Tacc>(st, rg.slots + (soff + node) * tsz, width);
            __syncthreads();
            if (tid == 0) {
                __threadfence();
                s_old = __hip_atomic_fetch_add(&rg.counters[coff + parent], 1, __ATOMIC_ACQ_REL,
                                               __HIP_MEMORY_SCOPE_AGENT);
                __threadfence();
            }
            __syncthreads();
            if (s_old != nchild - 1) return;  // the last child to arrive combines this node
            // R <- first child; absorb the others, stacked in child order.
            wg_load_tri<NP, Tacc>(st, rg.slots + (soff + first) * tsz, width);
            const RowSrc sib{rg.slots + (soff + first + 1) * tsz, nullptr, (int64_t)(nchild - 1) * width, NP, 0,
                             width};
            wg_absorb_rows<NP, double, Tacc, STAGED>(st, sib, 0, sib.rows_host, width, width);
        }
        node = parent;
        soff += n;
        coff += (n + A - 1) / A;
        n = (n + A - 1) / A;
    }
    wg_store<NP, Tacc>(st, rg.root, width);
}

template <int NP, typename Tin, typename Tacc, bool STAGED>
__global__ __launch_bounds__(64 * tree_waves(NP)) void k_tsqr_tree(TreeRegion reg0, TreeRegion reg1)
{
    const bool second = (int)blockIdx.x >= reg0.nleaves;
    tree_leaf<NP, Tin, Tacc, STAGED>(second ? reg1 : reg0, (int)blockIdx.x - (second ? reg0.nleaves : 0));
}

// The regions of a batch (device table): block b is leaf map[b].y of region map[b].x.
template <int NP, typename Tin, typename Tacc, bool STAGED>
__global__ __launch_bounds__(64 * tree_waves(NP)) void k_tsqr_tree_batch(const TreeRegion *__restrict__ regs,
                                                                         const int2 *__restrict__ map)
{
    const int2 e = map[blockIdx.x];
    const TreeRegion rg = regs[e.x];
    tree_leaf<NP, Tin, Tacc, STAGED>(rg, e.y);
}

// ------------------------------------------------------------------ one wave per triangle (tree)
//
// For launches with many more leaves than SIMDs (batches, long regions): each wave owns
// one triangle, so a column step needs no workgroup barrier and no LDS partial sums.
// With one row set per wave (NP = 64) the dot products are lane-local and the pivot
// column comes by lane reads; with several row sets the partial dots meet by lane swaps
// and the pivot column by a per-wave LDS slot.  The waves of a region then climb a tree
// of the region's arity as in the workgroup tree (per-node counters, last child combines
// the children in child order).

constexpr int kWtWaves = 4;  // independent waves per workgroup

// Absorb one block (RPT rows per lane in x) into the wave's triangle, columns [jstart, width).
template <int NP, typename Tacc>
__device__ inline void wt_block(Tacc (&x)[WaveGeom<NP>::RPT], Tacc *Rp, Tacc *xb, int k, int h, int jstart,
                                int width)
{
    constexpr int RPT = WaveGeom<NP>::RPT, H = WaveGeom<NP>::H;
    const bool col_ok = k < width;
    for (int j = jstart; j < width; j++) {
        const double alpha = (double)Rp[pidx(NP, j, j)];
        const Tacc rjk = Rp[pidx(NP, j, (k > j && col_ok) ? k : j)];
        Tacc xj[RPT];
        if constexpr (H == 1) {
#pragma unroll
            for (int i = 0; i < RPT; i++) xj[i] = readlane_t(x[i], j);
        } else {
            __builtin_amdgcn_wave_barrier();
            if (k == j) {
#pragma unroll
                for (int i = 0; i < RPT; i++) xb[i] = x[i];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int i = 0; i < RPT; i++) xj[i] = xb[i];
        }
        Tacc dp[8];
#pragma unroll
        for (int i = 0; i < 8; i++) dp[i] = xj[i] * x[i];
#pragma unroll
        for (int i = 8; i < RPT; i++) dp[i & 7] = fma(xj[i], x[i], dp[i & 7]);
        double d = (double)(((dp[0] + dp[1]) + (dp[2] + dp[3])) + ((dp[4] + dp[5]) + (dp[6] + dp[7])));
#pragma unroll
        for (int off = NP; off < 32; off <<= 1) d += __shfl_xor(d, off, 64);
        if constexpr (H >= 2) d = half_swap_sum(d);
        const double s = readlane_f64(d, j);
        const double q = fma(alpha, alpha, s);
        // A column whose norm is below the normal range is left untouched (tau = 0).
        const bool ok = s > 0.0 && q >= DBL_MIN;
        const double r = rsq_refined(ok ? q : 1.0);
        const double sg = alpha >= 0.0 ? 1.0 : -1.0;
        const double nrm = q * r;
        const double beta = -sg * nrm;
        const double inv_beta = -sg * r;
        const double scl = rcp_refined(ok ? alpha + sg * nrm : 1.0);
        const double tau = 1.0 - alpha * inv_beta;
        const double w = (double)rjk + scl * d;
        const bool upd = ok && k > j && col_ok;
        const Tacc c = upd ? (Tacc)(w * inv_beta) : Tacc(0);
        if (upd) {
#pragma unroll
            for (int i = 0; i < RPT; i++) x[i] += c * xj[i];
        }
        if (ok && h == 0 && k >= j && col_ok) Rp[pidx(NP, j, k)] = upd ? (Tacc)((double)rjk - tau * w) : (Tacc)beta;
    }
}

// Buffer-resource loads: one 32-bit offset register per load, and a load whose offset is
// at or past the resource's size returns 0.  (Descriptor word 3 of a raw 32-bit buffer on
// gfx9-family GPUs.)
constexpr int kBufWord3 = 0x00020000;

template <typename T>
__device__ inline T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ inline float buf_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
template <>
__device__ inline double buf_load<double>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

// Absorb rows [r0, r1) of src in blocks of BR rows.  tri_rows > 0: src is a stack of
// triangles of that many rows (a block inside one skips its known-zero columns).  Each
// block is read through a buffer resource that starts at its first row and ends at
// min(r1, block end): rows past r1 and columns outside the source (their offsets are set
// past the end) load as 0 with no branch or mask, so a block's loads are in flight
// together.  With FP32 accumulation the next block's loads are issued before the current
// block's column steps, which hide them.
template <int NP, typename Tin, typename Tacc, bool PREFETCH>
__device__ inline void wt_absorb_rows(Tacc *Rp, Tacc *xb, const RowSrc &src, int64_t r0, int64_t r1, int tri_rows,
                                      int width, int k, int h)
{
    constexpr int RPT = WaveGeom<NP>::RPT, BR = WaveGeom<NP>::BR;
    if (r0 >= r1) return;
    const int c = k - src.col_off;
    const bool col_in = k < width && c >= 0 && c < src.width;
    const uint32_t row_bytes = (uint32_t)(src.ld * (int64_t)sizeof(Tin));
    const uint32_t lane_off = (uint32_t)(((int64_t)h * RPT * src.ld + (c < 0 ? 0 : c)) * (int64_t)sizeof(Tin));
    auto load_rows = [&](Tacc (&y)[RPT], int64_t rb) {
        const uint32_t nrec = (uint32_t)(min(r1 - rb, (int64_t)BR) * (int64_t)row_bytes);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void *)((const char *)src.p + rb * (int64_t)row_bytes), (short)0, (int)nrec, kBufWord3);
        const uint32_t off = col_in ? lane_off : nrec;
#pragma unroll
        for (int i = 0; i < RPT; i++) y[i] = (Tacc)buf_load<Tin>(rs, off + (uint32_t)i * row_bytes);
    };
    Tacc xn[PREFETCH ? RPT : 1];
    if constexpr (PREFETCH) load_rows(xn, r0);
    for (int64_t rb = r0; rb < r1; rb += BR) {
        Tacc x[RPT];
        if constexpr (PREFETCH) {
#pragma unroll
            for (int i = 0; i < RPT; i++) x[i] = xn[i];
            if (rb + BR < r1) load_rows(xn, rb + BR);
        } else {
            load_rows(x, rb);
        }
        int jstart = src.col_off;
        if (tri_rows > 0) {
            const int64_t off = rb % tri_rows;
            if (off + BR <= tri_rows) jstart += (int)off;
        }
        wt_block<NP, Tacc>(x, Rp, xb, k, h, jstart, width);
    }
}

// ------------------------------------------------------------------ column-set layout (NP = 16, 32, 64)
//
// The wave as four row groups of 16 lanes: lane 16 g + p keeps columns p + 16 s (s < NS)
// of RPT rows of the block (rows g RPT .. g RPT + RPT - 1).  Column j sits in lane j % 16
// of every row group, so one lane permutation hands each group its own rows of the pivot
// column (no lane reads, no LDS writes); a dot product is a lane-local sum and two half
// swaps over the groups.  Column sets wholly left of the pivot are skipped, so the vector
// work of a step shrinks with the columns that remain.
// Rows per lane and set in a block (measured on the 256-instance batch): 16 at width 64
// (64-row blocks: the per-step reduction and reflector scalars are shared by twice the
// rows, worth more than the next block's loads in flight), 8 at width 128 (64 registers of
// X), otherwise 32 / NS with the next block prefetched into registers.
template <int NP>
struct SetGeom {
    static_assert(NP == 16 || NP == 32 || NP == 64 || NP == 128, "column-set layout");
    static constexpr int NS = NP / 16;                                       // column sets per lane
    static constexpr int RPT = NP == 64 ? 16 : (NP == 128 ? 8 : 32 / NS);  // rows per lane and set
    static constexpr int BR = 4 * RPT;                                       // rows per block
    static constexpr bool PREFETCH_OK = NS * RPT <= 32;  // registers for the next block
};

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// The value held by the lane at byte address `addr` (ds_bpermute: the LDS crossbar, no
// LDS memory).
__device__ __forceinline__ float lane_fetch(int addr, float v)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ double lane_fetch(int addr, double v)
{
    const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

// Half swaps of two registers (gfx950 v_permlane16_swap / v_permlane32_swap).  With rows
// of 16 lanes r0..r3: swap16(a, b) gives ([a.r0 b.r0 a.r2 b.r2], [a.r1 b.r1 a.r3 b.r3]) and
// swap32(a, b) gives ([a.r0 a.r1 b.r0 b.r1], [a.r2 a.r3 b.r2 b.r3]).
template <typename T>
struct Pair {
    T x, y;
};
__device__ __forceinline__ Pair<float> swap16(float a, float b)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return {__uint_as_float(r[0]), __uint_as_float(r[1])};
}
__device__ __forceinline__ Pair<float> swap32(float a, float b)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return {__uint_as_float(r[0]), __uint_as_float(r[1])};
}
__device__ __forceinline__ Pair<double> swap16(double a, double b)
{
    const auto l = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b), false,
                                                    false);
    const auto h = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false,
                                                    false);
    return {__hiloint2double((int)h[0], (int)l[0]), __hiloint2double((int)h[1], (int)l[1])};
}
__device__ __forceinline__ Pair<double> swap32(double a, double b)
{
    const auto l = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b), false,
                                                    false);
    const auto h = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false,
                                                    false);
    return {__hiloint2double((int)h[0], (int)l[0]), __hiloint2double((int)h[1], (int)l[1])};
}

// Sums over the four row groups of NA values at once (a[k]: this lane's partial of set k;
// entries k >= NA are ignored).  The result in row group g is the sum of set
// group_set<NA>(g): one set per group for NA = 3 or 4 (group 3 idle at 3), sets 0 1 0 1
// for NA = 2, set 0 everywhere for NA = 1.  Each group's sum adds the same partials in the
// same order in every lane that holds it.
template <int NA>
__device__ __forceinline__ int group_set(int g)
{
    return NA >= 3 ? g : (NA == 2 ? (g & 1) : 0);
}
template <int NA, typename T>
__device__ __forceinline__ T group_reduce(const T (&a)[4])
{
    if constexpr (NA == 1) {
        const Pair<T> u = swap16(a[0], a[0]);
        const T t = u.x + u.y;
        const Pair<T> v = swap32(t, t);
        return v.x + v.y;
    } else if constexpr (NA == 2) {
        const Pair<T> u = swap16(a[0], a[1]);
        const T t = u.x + u.y;
        const Pair<T> v = swap32(t, t);
        return v.x + v.y;
    } else {
        const Pair<T> u = swap16(a[0], a[1]);
        const Pair<T> w = swap16(a[2], NA == 4 ? a[3] : T(0));
        const Pair<T> v = swap32(u.x + u.y, w.x + w.y);
        return v.x + v.y;
    }
}
// The inverse: z holds, in group g, the value of set group_set<NA>(g); c[k] (k < NA) gets
// the value of set k in every lane.
template <int NA, typename T>
__device__ __forceinline__ void group_spread(T z, T (&c)[4])
{
    if constexpr (NA == 1) {
        c[0] = z;
    } else if constexpr (NA == 2) {
        const Pair<T> u = swap16(z, z);
        c[0] = u.x;
        c[1] = u.y;
    } else {
        const Pair<T> e = swap32(z, z);
        const Pair<T> u = swap16(e.x, e.x), v = swap16(e.y, e.y);
        c[0] = u.x;
        c[1] = u.y;
        c[2] = v.x;
        c[3] = v.y;
    }
}

// Reflector scalars in the accumulation type: FP64 with Newton-refined reciprocals, or
// FP32 with the hardware reciprocals (1 ulp) -- in an FP32 accumulation the dot products
// that feed them are FP32 sums already, so FP64 scalars buy neither range nor accuracy.
__device__ __forceinline__ double refl_rsq(double x) { return rsq_refined(x); }
__device__ __forceinline__ double refl_rcp(double x) { return rcp_refined(x); }
__device__ __forceinline__ float refl_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float refl_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double refl_min(double) { return DBL_MIN; }
__device__ __forceinline__ float refl_min(float) { return FLT_MIN; }

// Absorb one block (x[s][i]: column p + 16 s, row g RPT + i) into the wave's triangle,
// columns [jstart, width).  The reflector of wt_block, with its scalars in the
// accumulation type.  The pivot's column set S is a constant of each unrolled copy, so
// the sets it touches (NA = NS - S) are known at compile time.  They are taken in chunks
// of up to four: the dot products of a chunk's sets are summed over the row groups
// together, each group then finishes one set's column (w, the update coefficient, the new
// R entry) and the coefficients come back to every group by half swaps.
template <int NP, typename Tacc>
__device__ inline void ws_block(Tacc (&x)[SetGeom<NP>::NS][SetGeom<NP>::RPT], Tacc *Rp, int p, int g, int jstart,
                                int width)
{
    using Gm = SetGeom<NP>;
    constexpr int NS = Gm::NS, RPT = Gm::RPT;
    const int grp = (g * 16) << 2;  // byte address of this row group's lane 0
    static_for<0, NS>([&](auto sc) {
        constexpr int S = decltype(sc)::value, NA = NS - S, NC = (NA + 3) / 4;
        // per chunk: the column this row group finishes, and whether it writes it back
        // (one group per set)
        int col[NC];
        bool owns[NC];
        static_for<0, NC>([&](auto cc) {
            constexpr int C = decltype(cc)::value, NAC = NA - 4 * C < 4 ? NA - 4 * C : 4;
            const int gs = group_set<NAC>(g);
            owns[C] = g < NAC;
            col[C] = p + 16 * (S + 4 * C + (gs < NAC ? gs : 0));
        });
        const int j0 = max(jstart, 16 * S), j1 = min(width, 16 * S + 16);
        for (int j = j0; j < j1; j++) {
            const int jj = j - 16 * S;
            // Row j of R (only this step writes it, after these reads): issued first, so
            // that the LDS latency hides behind the dot products.  (For a column left of j
            // the read lands on an earlier entry of the packed triangle and is not used.)
            const Tacc alpha = Rp[pidx(NP, j, j)];
            Tacc *Rrow = Rp + (pidx(NP, j, j) - j);
            Tacc rjk[NC];
#pragma unroll
            for (int c = 0; c < NC; c++) rjk[c] = Rrow[col[c]];
            // this row group's rows of the pivot column
            Tacc piv[RPT];
#pragma unroll
            for (int i = 0; i < RPT; i++) piv[i] = lane_fetch(grp + (jj << 2), x[S][i]);
            Tacc d[NC];  // x_j . x_col for this group's column of each chunk
            static_for<0, NC>([&](auto cc) {
                constexpr int C = decltype(cc)::value, NAC = NA - 4 * C < 4 ? NA - 4 * C : 4;
                Tacc part[4];
#pragma unroll
                for (int k = 0; k < 4; k++) part[k] = Tacc(0);
#pragma unroll
                for (int k = 0; k < NAC; k++) {
                    const int sx = S + 4 * C + k;
                    Tacc a0 = piv[0] * x[sx][0], a1 = piv[1] * x[sx][1];
#pragma unroll
                    for (int i = 2; i < RPT; i += 2) {
                        a0 = fma(piv[i], x[sx][i], a0);
                        a1 = fma(piv[i + 1], x[sx][i + 1], a1);
                    }
                    part[k] = a0 + a1;
                }
                d[C] = group_reduce<NAC>(part);
            });
            const Tacc dj = readlane_t(d[0], jj);  // group 0 finishes set S, pivot lane jj
            const Tacc q = fma(alpha, alpha, dj);
            // A column whose norm is below the normal range is left untouched (tau = 0).
            const bool ok = dj > Tacc(0) && q >= refl_min(q);
            const Tacc r = refl_rsq(ok ? q : Tacc(1));
            const Tacc sg = alpha >= Tacc(0) ? Tacc(1) : Tacc(-1);
            const Tacc nrm = q * r;
            const Tacc beta = -sg * nrm;
            const Tacc inv_beta = -sg * r;
            const Tacc scl = refl_rcp(ok ? alpha + sg * nrm : Tacc(1));
            const Tacc tau = Tacc(1) - alpha * inv_beta;
            static_for<0, NC>([&](auto cc) {
                constexpr int C = decltype(cc)::value, NAC = NA - 4 * C < 4 ? NA - 4 * C : 4;
                const bool upd = ok && col[C] > j && col[C] < width;
                const Tacc w = fma(scl, d[C], rjk[C]);
                if (ok && owns[C] && col[C] >= j && col[C] < width) Rrow[col[C]] = upd ? fma(-tau, w, rjk[C]) : beta;
                // c = 0 leaves a column as it is (no branch around the update)
                Tacc cf[4];
                group_spread<NAC>(upd ? w * inv_beta : Tacc(0), cf);
#pragma unroll
                for (int k = 0; k < NAC; k++)
#pragma unroll
                    for (int i = 0; i < RPT; i++) x[S + 4 * C + k][i] = fma(cf[k], piv[i], x[S + 4 * C + k][i]);
            });
        }
    });
}

// Rows of a block of the wave tree's leaves.
template <int NP>
__host__ __device__ constexpr int wave_leaf_rows()
{
    if constexpr (NP >= 16)
        return SetGeom<NP>::BR;
    else
        return WaveGeom<NP>::BR;
}

// wt_absorb_rows for the column-set layout.
template <int NP, typename Tin, typename Tacc, bool PREFETCH>
__device__ inline void ws_absorb_rows(Tacc *Rp, const RowSrc &src, int64_t r0, int64_t r1, int tri_rows, int width,
                                      int p, int g)
{
    using Gm = SetGeom<NP>;
    constexpr int NS = Gm::NS, RPT = Gm::RPT, BR = Gm::BR;
    if (r0 >= r1) return;
    const uint32_t row_bytes = (uint32_t)(src.ld * (int64_t)sizeof(Tin));
    uint32_t loff[NS];
    bool col_in[NS];
#pragma unroll
    for (int s = 0; s < NS; s++) {
        const int c = p + 16 * s - src.col_off;
        col_in[s] = p + 16 * s < width && c >= 0 && c < src.width;
        loff[s] = (uint32_t)(((int64_t)g * RPT * src.ld + (c < 0 ? 0 : c)) * (int64_t)sizeof(Tin));
    }
    auto load_rows = [&](Tacc (&y)[NS][RPT], int64_t rb) {
        const uint32_t nrec = (uint32_t)(min(r1 - rb, (int64_t)BR) * (int64_t)row_bytes);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void *)((const char *)src.p + rb * (int64_t)row_bytes), (short)0, (int)nrec, kBufWord3);
#pragma unroll
        for (int s = 0; s < NS; s++) {
            const uint32_t off = col_in[s] ? loff[s] : nrec;
#pragma unroll
            for (int i = 0; i < RPT; i++) y[s][i] = (Tacc)buf_load<Tin>(rs, off + (uint32_t)i * row_bytes);
        }
    };
    Tacc xn[PREFETCH ? NS : 1][PREFETCH ? RPT : 1];
    if constexpr (PREFETCH) load_rows(xn, r0);
    for (int64_t rb = r0; rb < r1; rb += BR) {
        Tacc x[NS][RPT];
        if constexpr (PREFETCH) {
#pragma unroll
            for (int s = 0; s < NS; s++)
#pragma unroll
                for (int i = 0; i < RPT; i++) x[s][i] = xn[s][i];
            if (rb + BR < r1) load_rows(xn, rb + BR);
        } else {
            load_rows(x, rb);
        }
        int jstart = src.col_off;
        if (tri_rows > 0) {
            const int64_t off = rb % tri_rows;
            if (off + BR <= tri_rows) jstart += (int)off;
        }
        ws_block<NP, Tacc>(x, Rp, p, g, jstart, width);
    }
}

template <int NP, typename Tacc>
__device__ inline void wt_load_tri(Tacc *Rp, const double *T, int width, int lane)
{
    for (int e = lane; e < WaveGeom<NP>::PS; e += 64) Rp[e] = Tacc(0);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (T) {
        staged_copy<8, double>(
            width * NP, lane, 64, [&](int e) { return T[e]; },
            [&](int e, double v) {
                const int j = e / NP, kk = e - j * NP;
                if (kk >= j && kk < width) Rp[pidx(NP, j, kk)] = (Tacc)v;
            });
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// A value the whole wave holds (read from lane 0), so that the compiler keeps it and
// everything derived from it in scalar registers.
__device__ inline int64_t wave_uniform(int64_t v)
{
    const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Leaf g of region rg by one wave, then the climb of its tree.
template <int NP, typename Tin, typename Tacc>
__device__ __forceinline__ void wt_leaf(const TreeRegion &rg, const int g, Tacc *Rp, Tacc *xbase, int lane)
{
    using Gm = WaveGeom<NP>;
    const int k = lane % NP, h = lane / NP;
    Tacc *xb = xbase + h * Gm::RPT;
    const int width = rg.width;
    const int64_t rows = wave_uniform(src_rows(rg.src));
    const int64_t want = (rows + rg.rows_per_leaf - 1) / rg.rows_per_leaf;
    const int nleaves = (int)max((int64_t)1, min((int64_t)rg.nleaves, want));
    if (g >= nleaves) return;
    wt_load_tri<NP, Tacc>(Rp, nullptr, width, lane);
    int64_t chunk = (rows + nleaves - 1) / nleaves;
    constexpr int LBR = wave_leaf_rows<NP>();
    chunk = ((chunk + LBR - 1) / LBR) * LBR;
    const int64_t r0 = (int64_t)g * chunk, r1 = min(rows, r0 + chunk);
    if constexpr (NP >= 16)
        ws_absorb_rows<NP, Tin, Tacc, sizeof(Tacc) == 4 && SetGeom<NP>::PREFETCH_OK>(Rp, rg.src, r0, r1, 0, width,
                                                                                   lane & 15, lane >> 4);
    else
        wt_absorb_rows<NP, Tin, Tacc, sizeof(Tacc) == 4>(Rp, xb, rg.src, r0, r1, 0, width, k, h);

    const int64_t tsz = (int64_t)width * NP;
    const int A = rg.arity;
    int node = g, n = nleaves;
    int64_t soff = 0, coff = 0;
    while (n > 1) {
        const int parent = node / A, first = parent * A;
        const int nchild = min(A, n - first);
        if (nchild > 1) {
            wave_store<NP, Tacc>(Rp, rg.slots + (soff + node) * tsz, width, lane);
            __threadfence();
            int old = 0;
            if (lane == 0)
                old = __hip_atomic_fetch_add(&rg.counters[coff + parent], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            old = __builtin_amdgcn_readfirstlane(old);  // lane 0's value, uniform in the wave
            if (old != nchild - 1) return;  // the last child to arrive combines this node
            __threadfence();
            // R <- first child; absorb the others, stacked in child order.
            wt_load_tri<NP, Tacc>(Rp, rg.slots + (soff + first) * tsz, width, lane);
            const RowSrc sib{rg.slots + (soff + first + 1) * tsz, nullptr, (int64_t)(nchild - 1) * width, NP, 0,
                             width};
            if constexpr (NP >= 16)
                ws_absorb_rows<NP, double, Tacc, false>(Rp, sib, 0, sib.rows_host, width, width, lane & 15, lane >> 4);
            else
                wt_absorb_rows<NP, double, Tacc, false>(Rp, xb, sib, 0, sib.rows_host, width, width, k, h);
        }
        node = parent;
        soff += n;
        coff += (n + A - 1) / A;
        n = (n + A - 1) / A;
    }
    wave_store<NP, Tacc>(Rp, rg.root, width, lane);
}

// The regions of a batch by waves (device table): wave item of the grid is leaf map[item].y
// of region map[item].x; surplus waves of the last workgroup leave at once (no workgroup
// barrier follows).
template <int NP, typename Tin, typename Tacc>
__global__ __launch_bounds__(64 * kWtWaves) void k_tsqr_wtree_batch(const TreeRegion *__restrict__ regs,
                                                                    const int2 *__restrict__ map, int64_t nitems)
{
    using Gm = WaveGeom<NP>;
    __shared__ Tacc Rs[kWtWaves][Gm::PS];
    __shared__ __align__(16) Tacc Xs[kWtWaves][Gm::BR];
    // the wave index is uniform in each wave; say so, so that everything derived from it
    // (the item, its region descriptor, the buffer resources) lives in scalar registers
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t item = (int64_t)blockIdx.x * kWtWaves + wv;
    if (item >= nitems) return;
    const int2 e = map[item];
    const TreeRegion rg = regs[e.x];
    wt_leaf<NP, Tin, Tacc>(rg, e.y, Rs[wv], Xs[wv], lane);
}

// Every narrow width of a batch in one launch: wave item i is leaf map[i].y of region
// map[i].x, of padded width map[i].z (the map lists the widest leaves first, so that the
// longest leaves start first and the narrower ones fill the compute units as the wide
// ones drain).  Each wave's LDS slice holds its triangle and then its row buffer, carved
// for its own width: the slice of the widest width, as in the single-width kernel.
__host__ __device__ constexpr int wt_slice_tri(int np) { return (packed_size(np) + 3) / 4 * 4; }
constexpr int kWtSlice = wt_slice_tri(64) + 32;  // the largest of wt_slice_tri(np) + rows of a block
static_assert(kWtSlice >= wt_slice_tri(32) + 64 && kWtSlice >= wt_slice_tri(16) + 128 &&
                  kWtSlice >= wt_slice_tri(8) + 256 && kWtSlice >= wt_slice_tri(4) + 512,
              "wave slice");

// At least four waves per SIMD (measured on the 256-instance batch, FP32: 2.19 ms against
// 2.37 ms at three; the few values the compiler spills for it sit outside the column steps).
template <typename Tin, typename Tacc>
__global__ __launch_bounds__(64 * kWtWaves, 4) void k_tsqr_wtree_multi(const TreeRegion *__restrict__ regs,
                                                                    const int4 *__restrict__ map, int64_t nitems)
{
    __shared__ __align__(16) Tacc Ls[kWtWaves][kWtSlice];
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t item = (int64_t)blockIdx.x * kWtWaves + wv;
    if (item >= nitems) return;
    const int4 e = map[item];
    const TreeRegion rg = regs[e.x];
    Tacc *sl = Ls[wv];
    switch (__builtin_amdgcn_readfirstlane(e.z)) {
    case 64: wt_leaf<64, Tin, Tacc>(rg, e.y, sl, sl + wt_slice_tri(64), lane); break;
    case 32: wt_leaf<32, Tin, Tacc>(rg, e.y, sl, sl + wt_slice_tri(32), lane); break;
    case 16: wt_leaf<16, Tin, Tacc>(rg, e.y, sl, sl + wt_slice_tri(16), lane); break;
    case 8: wt_leaf<8, Tin, Tacc>(rg, e.y, sl, sl + wt_slice_tri(8), lane); break;
    case 4: wt_leaf<4, Tin, Tacc>(rg, e.y, sl, sl + wt_slice_tri(4), lane); break;
    default: break;
    }
}

__global__ void k_sign_normalise(const double *Rin, int64_t ldin, int n, double *R, int64_t ldr)
{
    // one wave per row
    const int i = blockIdx.x;
    const int lane = threadIdx.x;
    const double *row = Rin + (int64_t)i * ldin;
    const double d = row[i];
    bool neg = d < 0.0;
    if (d == 0.0) {
        // first nonzero entry at or right of the diagonal decides
        int first = n;
        for (int k = i + lane; k < n; k += 64) {
            if (row[k] != 0.0) { first = k; break; }
        }
        for (int off = 32; off > 0; off >>= 1) first = min(first, __shfl_xor(first, off, 64));
        neg = first < n && row[first] < 0.0;
    }
    for (int k = lane; k < n; k += 64) {
        double v = (k < i) ? 0.0 : (neg ? -row[k] : row[k]);
        R[(int64_t)i * ldr + k] = v + 0.0;
    }
}

template <int NP>
hipError_t launch_np(int acc_f64, int in_f64, const double *init, int64_t init_ld, RowSrc s0,
                     RowSrc s1, int nsrc, int width, int tri_rows, int nwg, double *tri,
                     int64_t stride, hipStream_t s)
{
    if constexpr (NP <= 64) {
        const unsigned grid = (unsigned)((nwg + kWavesPerBlock - 1) / kWavesPerBlock);
#define FIGARO_WAVE(TI, TA)                                                                    \
    k_tsqr_wave<NP, TI, TA><<<grid, 64 * kWavesPerBlock, 0, s>>>(init, init_ld, s0, s1, nsrc,  \
                                                                 width, tri_rows, nwg, tri, stride)
        if (acc_f64) {
            if (in_f64) FIGARO_WAVE(double, double);
            else FIGARO_WAVE(float, double);
        } else {
            if (in_f64) FIGARO_WAVE(double, float);
            else FIGARO_WAVE(float, float);
        }
#undef FIGARO_WAVE
        return hipGetLastError();
    } else {
        return launch_tsqr_panel(NP, acc_f64, in_f64, init, init_ld, s0, s1, nsrc, width, tri_rows, nwg, tri,
                                 stride, s);
    }
}

template <int NP>
hipError_t launch_tree_np(int acc_f64, int in_f64, const TreeRegion *regs, int nreg, hipStream_t s)
{
    TreeRegion r0 = regs[0];
    TreeRegion r1 = nreg > 1 ? regs[1] : TreeRegion{};
    const unsigned grid = (unsigned)(r0.nleaves + r1.nleaves);
    // at most one leaf per compute unit: staged loads (see wg_absorb_rows)
    const bool staged = grid <= 256;
#define FIGARO_TREE(TI, TA)                                                                   \
    do {                                                                                      \
        if (staged) k_tsqr_tree<NP, TI, TA, true><<<grid, 64 * tree_waves(NP), 0, s>>>(r0, r1);  \
        else k_tsqr_tree<NP, TI, TA, false><<<grid, 64 * tree_waves(NP), 0, s>>>(r0, r1);        \
    } while (0)
    if (acc_f64) {
        if (in_f64) FIGARO_TREE(double, double);
        else FIGARO_TREE(float, double);
    } else {
        if (in_f64) FIGARO_TREE(double, float);
        else FIGARO_TREE(float, float);
    }
#undef FIGARO_TREE
    return hipGetLastError();
}

// One or two regions by waves (a single call): wave item i < reg0.nleaves is leaf i of
// region 0, the rest leaves of region 1.
// ------------------------------------------------------------------ Givens rotations (one wave per triangle)
//
// The continuation of Claim 1 entry by entry (Section 1): each new row x is absorbed
// into R by plane rotations, column by column: the rotation of (R_jj, x_j) that zeroes
// x_j touches row j of R and x only, and leaves zeros where they are.  Lane k holds
// column k of R (row j in r[j], the loop over j unrolled so every index is static) and
// entry k of the current row; the two scalars of step j come from lane j by lane reads.
// R keeps a non-negative diagonal throughout (R_jj <- |(R_jj, x_j)|).  FP64.

// Absorb rows [r0, r1) of src (one row at a time, the next row's load issued before the
// current row's rotations).
template <int NP, typename Tin>
__device__ inline void gv_absorb_rows(double (&r)[NP], const RowSrc &src, int64_t r0, int64_t r1, int width, int k)
{
    const int c = k - src.col_off;
    const bool col_in = k < width && c >= 0 && c < src.width;
    const Tin *col = (const Tin *)src.p + (c < 0 ? 0 : (c < src.width ? c : src.width - 1));
    if (r0 >= r1) return;
    double xn = (double)col[r0 * src.ld];
    for (int64_t row = r0; row < r1; row++) {
        double x = col_in ? xn : 0.0;
        if (row + 1 < r1) xn = (double)col[(row + 1) * src.ld];
#pragma unroll
        for (int j = 0; j < NP; j++) {
            const double a = readlane_f64(r[j], j), b = readlane_f64(x, j);
            const double q = fma(a, a, b * b);
            // (columns past the width hold zeros: b = 0 leaves them alone)
            if (b != 0.0 && q >= DBL_MIN) {
                const double inv = rsq_refined(q);
                const double cs = a * inv, sn = b * inv;
                if (k > j) {
                    const double rj = r[j];
                    r[j] = fma(cs, rj, sn * x);
                    x = fma(cs, x, -sn * rj);
                } else if (k == j) {
                    r[j] = q * inv;
                    x = 0.0;
                }
            }
        }
    }
}

template <int NP>
__device__ inline void gv_store(const double (&r)[NP], double *out, int width, int k)
{
#pragma unroll
    for (int j = 0; j < NP; j++)
        if (j < width && k < NP) out[(int64_t)j * NP + k] = (k >= j && k < width) ? r[j] : 0.0;
}

// Leaf g of region rg by one wave (rows by rotations), then the climb of its tree (the
// last child absorbs its siblings' triangles, row by row, in child order).
template <int NP, typename Tin>
__device__ __forceinline__ void gv_leaf(const TreeRegion &rg, const int g, int lane)
{
    const int k = lane;
    const int width = rg.width;
    const int64_t rows = wave_uniform(src_rows(rg.src));
    const int64_t want = (rows + rg.rows_per_leaf - 1) / rg.rows_per_leaf;
    const int nleaves = (int)max((int64_t)1, min((int64_t)rg.nleaves, want));
    if (g >= nleaves) return;
    double r[NP];
#pragma unroll
    for (int j = 0; j < NP; j++) r[j] = 0.0;
    const int64_t chunk = (rows + nleaves - 1) / nleaves;
    const int64_t r0 = (int64_t)g * chunk, r1 = min(rows, r0 + chunk);
    gv_absorb_rows<NP, Tin>(r, rg.src, r0, r1, width, k);
    const int64_t tsz = (int64_t)width * NP;
    const int A = rg.arity;
    int node = g, n = nleaves;
    int64_t soff = 0, coff = 0;
    while (n > 1) {
        const int parent = node / A, first = parent * A;
        const int nchild = min(A, n - first);
        if (nchild > 1) {
            gv_store<NP>(r, rg.slots + (soff + node) * tsz, width, k);
            __threadfence();
            int old = 0;
            if (lane == 0)
                old = __hip_atomic_fetch_add(&rg.counters[coff + parent], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            old = __builtin_amdgcn_readfirstlane(old);
            if (old != nchild - 1) return;  // the last child to arrive combines this node
            __threadfence();
            const double *T = rg.slots + (soff + first) * tsz;
#pragma unroll
            for (int j = 0; j < NP; j++) r[j] = (j < width && k < width) ? T[(int64_t)j * NP + k] : 0.0;
            const RowSrc sib{rg.slots + (soff + first + 1) * tsz, nullptr, (int64_t)(nchild - 1) * width, NP, 0,
                             width};
            gv_absorb_rows<NP, double>(r, sib, 0, sib.rows_host, width, k);
        }
        node = parent;
        soff += n;
        coff += (n + A - 1) / A;
        n = (n + A - 1) / A;
    }
    gv_store<NP>(r, rg.root, width, k);
}

// One or two regions by rotations: wave item i < reg0.nleaves is leaf i of region 0,
// the rest leaves of region 1.
template <int NP, typename Tin>
__global__ __launch_bounds__(64 * kWtWaves) void k_givens_tree(TreeRegion reg0, TreeRegion reg1)
{
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int item = (int)blockIdx.x * kWtWaves + wv;
    if (item >= reg0.nleaves + reg1.nleaves) return;
    const bool second = item >= reg0.nleaves;
    gv_leaf<NP, Tin>(second ? reg1 : reg0, item - (second ? reg0.nleaves : 0), lane);
}

template <int NP, typename Tin, typename Tacc>
__global__ __launch_bounds__(64 * kWtWaves) void k_tsqr_wtree(TreeRegion reg0, TreeRegion reg1)
{
    using Gm = WaveGeom<NP>;
    __shared__ Tacc Rs[kWtWaves][Gm::PS];
    __shared__ __align__(16) Tacc Xs[kWtWaves][Gm::BR];
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int item = (int)blockIdx.x * kWtWaves + wv;
    if (item >= reg0.nleaves + reg1.nleaves) return;
    const bool second = item >= reg0.nleaves;
    wt_leaf<NP, Tin, Tacc>(second ? reg1 : reg0, item - (second ? reg0.nleaves : 0), Rs[wv], Xs[wv], lane);
}

// Padded width 128: one wave per workgroup (its packed triangle takes 33 KB of LDS in
// FP32, 66 KB in FP64).
template <typename Tin, typename Tacc>
__global__ __launch_bounds__(64) void k_tsqr_wtree128(TreeRegion reg0, TreeRegion reg1)
{
    __shared__ Tacc Rs[WaveGeom<128>::PS];
    const int lane = threadIdx.x;
    const int item = (int)blockIdx.x;
    if (item >= reg0.nleaves + reg1.nleaves) return;
    const bool second = item >= reg0.nleaves;
    wt_leaf<128, Tin, Tacc>(second ? reg1 : reg0, item - (second ? reg0.nleaves : 0), Rs, Rs, lane);
}

hipError_t launch_wtree128(int acc_f64, int in_f64, const TreeRegion *regs, int nreg, hipStream_t s)
{
    TreeRegion r0 = regs[0];
    TreeRegion r1 = nreg > 1 ? regs[1] : TreeRegion{};
    const unsigned grid = (unsigned)(r0.nleaves + r1.nleaves);
#define FIGARO_TREE(TI, TA) k_tsqr_wtree128<TI, TA><<<grid, 64, 0, s>>>(r0, r1)
    if (acc_f64) {
        if (in_f64) FIGARO_TREE(double, double);
        else FIGARO_TREE(float, double);
    } else {
        if (in_f64) FIGARO_TREE(double, float);
        else FIGARO_TREE(float, float);
    }
#undef FIGARO_TREE
    return hipGetLastError();
}

template <int NP>
hipError_t launch_wtree_np(int acc_f64, int in_f64, const TreeRegion *regs, int nreg, hipStream_t s)
{
    TreeRegion r0 = regs[0];
    TreeRegion r1 = nreg > 1 ? regs[1] : TreeRegion{};
    const unsigned grid = (unsigned)((r0.nleaves + r1.nleaves + kWtWaves - 1) / kWtWaves);
#define FIGARO_TREE(TI, TA) k_tsqr_wtree<NP, TI, TA><<<grid, 64 * kWtWaves, 0, s>>>(r0, r1)
    if (acc_f64) {
        if (in_f64) FIGARO_TREE(double, double);
        else FIGARO_TREE(float, double);
    } else {
        if (in_f64) FIGARO_TREE(double, float);
        else FIGARO_TREE(float, float);
    }
#undef FIGARO_TREE
    return hipGetLastError();
}

template <int NP>
hipError_t launch_tree_batch_np(int wave_tree, int acc_f64, int in_f64, const TreeRegion *regs, const int2 *map,
                                int64_t nitems, hipStream_t s)
{
    const unsigned grid = (unsigned)(wave_tree ? (nitems + kWtWaves - 1) / kWtWaves : nitems);
#define FIGARO_TREE(TI, TA)                                                                              \
    do {                                                                                                 \
        if (wave_tree) k_tsqr_wtree_batch<NP, TI, TA><<<grid, 64 * kWtWaves, 0, s>>>(regs, map, nitems);  \
        else k_tsqr_tree_batch<NP, TI, TA, false><<<grid, 64 * tree_waves(NP), 0, s>>>(regs, map);        \
    } while (0)
    if (acc_f64) {
        if (in_f64) FIGARO_TREE(double, double);
        else FIGARO_TREE(float, double);
    } else {
        if (in_f64) FIGARO_TREE(double, float);
        else FIGARO_TREE(float, float);
    }
#undef FIGARO_TREE
    return hipGetLastError();
}

}  // namespace

hipError_t launch_tsqr_tree_batch(int wave_tree, int np, int acc_f64, int in_f64, const TreeRegion *regs,
                                  const int2 *map, int64_t nitems, hipStream_t s)
{
    if (nitems == 0) return hipSuccess;
    if (nitems > INT32_MAX) return hipErrorInvalidValue;
    switch (np) {
#define FIGARO_CASE(NPV) \
    case NPV: return launch_tree_batch_np<NPV>(wave_tree, acc_f64, in_f64, regs, map, nitems, s);
    FIGARO_CASE(4) FIGARO_CASE(8) FIGARO_CASE(16) FIGARO_CASE(32) FIGARO_CASE(64)
#undef FIGARO_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_tsqr_wtree_multi(int acc_f64, int in_f64, const TreeRegion *regs, const int4 *map, int64_t nitems,
                                   hipStream_t s)
{
    if (nitems == 0) return hipSuccess;
    if (nitems > INT32_MAX) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)((nitems + kWtWaves - 1) / kWtWaves);
#define FIGARO_MULTI(TI, TA) k_tsqr_wtree_multi<TI, TA><<<grid, 64 * kWtWaves, 0, s>>>(regs, map, nitems)
    if (acc_f64) {
        if (in_f64) FIGARO_MULTI(double, double);
        else FIGARO_MULTI(float, double);
    } else {
        if (in_f64) FIGARO_MULTI(double, float);
        else FIGARO_MULTI(float, float);
    }
#undef FIGARO_MULTI
    return hipGetLastError();
}

int tsqr_padded_width(int n)
{
    if (n <= 0) return 0;
    int np = 4;
    while (np < n) np <<= 1;
    return np <= 512 ? np : 0;
}

int tsqr_block_rows(int np, int acc_f64)
{
    if (np <= 64) return tree_waves(np) * wave_block_rows(np);  // tree kernel: waves x row sets x rows per lane
    return tsqr_panel_rows(np, acc_f64);                   // workgroup panel kernel
}

int tsqr_wave_block_rows(int np)
{
    switch (np) {
    case 16: return wave_leaf_rows<16>();
    case 32: return wave_leaf_rows<32>();
    case 64: return wave_leaf_rows<64>();
    case 128: return wave_leaf_rows<128>();
    default: return wave_block_rows(np);
    }
}

int tsqr_tree_arity(int np, int width)
{
    const int a = 1 + tree_waves(np) * wave_block_rows(np) / (width > 0 ? width : 1);
    return a < 2 ? 2 : (a > 32 ? 32 : a);
}

void tsqr_tree_sizes(int nleaves, int arity, int64_t *slots, int64_t *counters)
{
    int64_t s = 0, c = 0;
    int n = nleaves;
    while (n > 1) {
        s += n;
        c += (n + arity - 1) / arity;
        n = (n + arity - 1) / arity;
    }
    *slots = s + 1;
    *counters = c + 1;
}

hipError_t launch_tsqr_stream(int np, int acc_f64, int in_f64, const double *init, int64_t init_ld,
                              RowSrc s0, RowSrc s1, int nsrc, int width, int tri_rows, int nwg,
                              double *tri, int64_t tri_stride, hipStream_t s)
{
    switch (np) {
#define FIGARO_CASE(NPV) \
    case NPV: return launch_np<NPV>(acc_f64, in_f64, init, init_ld, s0, s1, nsrc, width, tri_rows, nwg, tri, tri_stride, s);
    FIGARO_CASE(4) FIGARO_CASE(8) FIGARO_CASE(16) FIGARO_CASE(32) FIGARO_CASE(64) FIGARO_CASE(128) FIGARO_CASE(256)
    FIGARO_CASE(512)
#undef FIGARO_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_givens_tree(int np, int in_f64, const TreeRegion *regs, int nreg, hipStream_t s)
{
    if (nreg < 1 || nreg > 2) return hipErrorInvalidValue;
    TreeRegion r0 = regs[0];
    TreeRegion r1 = nreg > 1 ? regs[1] : TreeRegion{};
    const unsigned grid = (unsigned)((r0.nleaves + r1.nleaves + kWtWaves - 1) / kWtWaves);
    switch (np) {
#define FIGARO_CASE(NPV)                                                                      \
    case NPV:                                                                                 \
        if (in_f64) k_givens_tree<NPV, double><<<grid, 64 * kWtWaves, 0, s>>>(r0, r1);       \
        else k_givens_tree<NPV, float><<<grid, 64 * kWtWaves, 0, s>>>(r0, r1);               \
        return hipGetLastError();
    FIGARO_CASE(4) FIGARO_CASE(8) FIGARO_CASE(16) FIGARO_CASE(32) FIGARO_CASE(64)
#undef FIGARO_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_tsqr_tree(int np, int acc_f64, int in_f64, const TreeRegion *regs, int nreg,
                            hipStream_t s, int wave_tree)
{
    if (nreg < 1 || nreg > 2) return hipErrorInvalidValue;
    switch (np) {
#define FIGARO_CASE(NPV) \
    case NPV: return wave_tree ? launch_wtree_np<NPV>(acc_f64, in_f64, regs, nreg, s) \
                               : launch_tree_np<NPV>(acc_f64, in_f64, regs, nreg, s);
    FIGARO_CASE(4) FIGARO_CASE(8) FIGARO_CASE(16) FIGARO_CASE(32) FIGARO_CASE(64)
#undef FIGARO_CASE
    case 128:
        // the workgroup kernel of this width is the streaming panel tree
        return wave_tree ? launch_wtree128(acc_f64, in_f64, regs, nreg, s)
                         : launch_tsqr_panel_tree(128, acc_f64, in_f64, regs, nreg, s);
    default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------ Cartesian root
//
// The root of the two-sided form of a Cartesian product in one wave.  R starts as
// diag(R_TA, R_TB) (the upper triangles of the two tails' roots, widths na and nb) and
// absorbs the single head row h = [sqrt(m2) H(A) | sqrt(m1) H(B)] of the one group.
// With one row, the reflector of column j acts on the pair (R_jj, h_j) only: a plane
// rotation that zeroes h_j and rotates row j of R with h.  It leaves rows j+1.. of R
// untouched, so row j+1 is read from LDS while step j runs.  Lane l owns columns
// l + 64 c (one for NP <= 64, two for NP = 128) and keeps its entries of h and of the
// current row of R in registers; the two scalars of a step come from lane j by lane
// reads.  The packed triangle lives in LDS (66 KB at NP = 128).  R is written out with
// every row's sign normalised (diagonal >= 0; a zero diagonal takes the sign of the row's
// first nonzero entry; -0.0 becomes +0.0).  With no group (an empty table) nothing is
// absorbed.
template <int NP>
__device__ __forceinline__ void merge_cartesian_lds(const double *Ta, int64_t lda, int na, const double *Tb,
                                                    int64_t ldb, int nb, Groups g, const double *hA,
                                                    const double *hB, double *R, int64_t ldr)
{
    constexpr int CPL = NP > 64 ? NP / 64 : 1;
    __shared__ double Rp[packed_size(NP)];
    const int lane = threadIdx.x, width = na + nb;
    // diag(Ta, Tb) into the packed triangle; every load is clamped into its source
    staged_copy<16, double>(
        width * NP, lane, 64,
        [&](int e) {
            // base pointer and clamped offset chosen first: one unconditional load
            const int j = e / NP, kk = e - j * NP;
            const bool top = j < na;
            const double *p = top ? Ta + (int64_t)j * lda : Tb + (int64_t)(j - na) * ldb;
            const int c = top ? (kk < na ? kk : na - 1) : (kk < na ? 0 : (kk < width ? kk - na : nb - 1));
            return p[c];
        },
        [&](int e, double v) {
            const int j = e / NP, kk = e - j * NP;
            if (kk < j) return;
            const bool in = j < na ? kk < na : (kk >= na && kk < width);
            Rp[pidx(NP, j, kk)] = in ? v : 0.0;
        });
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (g.counts[CNT_G] > 0) {
        const double s2 = sqrt((double)g.m2[0]), s1 = sqrt((double)g.m1[0]);
        double h[CPL], rj[CPL];
#pragma unroll
        for (int c = 0; c < CPL; c++) {
            const int col = lane + 64 * c;
            h[c] = col < na ? s2 * hA[col] : (col < width ? s1 * hB[col - na] : 0.0);
            rj[c] = col < width ? Rp[pidx(NP, 0, col)] : 0.0;
        }
        for (int j = 0; j < width; j++) {
            double rn[CPL];  // row j + 1 of R, which step j does not change
#pragma unroll
            for (int c = 0; c < CPL; c++) {
                const int col = lane + 64 * c;
                rn[c] = (col > j && col < width) ? Rp[pidx(NP, j + 1, col)] : 0.0;
            }
            double alpha = 0.0, hj = 0.0;
#pragma unroll
            for (int c = 0; c < CPL; c++)
                if (j / 64 == c) {
                    alpha = readlane_f64(rj[c], j % 64);
                    hj = readlane_f64(h[c], j % 64);
                }
            const double q = fma(alpha, alpha, hj * hj);
            if (hj != 0.0 && q >= DBL_MIN) {
                const double rinv = rsq_refined(q);
                const double cs = alpha * rinv, sn = hj * rinv;
#pragma unroll
                for (int c = 0; c < CPL; c++) {
                    const int col = lane + 64 * c;
                    if (col > j && col < width) {
                        const double a = rj[c], b = h[c];
                        Rp[pidx(NP, j, col)] = fma(cs, a, sn * b);
                        h[c] = fma(cs, b, -sn * a);
                    } else if (col == j) {
                        Rp[pidx(NP, j, j)] = q * rinv;
                        h[c] = 0.0;
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < CPL; c++) rj[c] = rn[c];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int i = 0; i < width; i++) {
        const double d = Rp[pidx(NP, i, i)];
        bool neg = d < 0.0;
        if (d == 0.0) {
            int first = width;
            for (int k = i + lane; k < width; k += 64)
                if (Rp[pidx(NP, i, k)] != 0.0) {
                    first = k;
                    break;
                }
            for (int off = 32; off > 0; off >>= 1) first = min(first, __shfl_xor(first, off, 64));
            neg = first < width && Rp[pidx(NP, i, first)] < 0.0;
        }
        for (int k = lane; k < width; k += 64) {
            const double v = k < i ? 0.0 : Rp[pidx(NP, i, k)];
            R[(int64_t)i * ldr + k] = (neg ? -v : v) + 0.0;
        }
    }
}

// The same for NP <= 64 with R in registers: lane k holds column k of R (row j in r[j]),
// and the column loop is unrolled so that every row index is static.  No LDS: the two
// scalars of step j come from lane j by lane reads, and row i is written out by the
// lanes straight from r[i].
template <int NP>
__device__ __forceinline__ void merge_cartesian_reg(const double *Ta, int64_t lda, int na, const double *Tb,
                                                    int64_t ldb, int nb, Groups g, const double *hA,
                                                    const double *hB, double *R, int64_t ldr)
{
    static_assert(NP <= 64, "one column per lane");
    const int k = threadIdx.x, width = na + nb;
    const bool col_ok = k < width;
    // column k of diag(Ta, Tb): rows of Ta for k < na, rows of Tb below them otherwise
    // (clamped loads: every address lies inside its triangle)
    double r[NP];
    const int kc = k < width ? k : width - 1;
    const bool top = kc < na;
    // one base pointer and stride per lane, so that every load is unconditional (a select
    // between two loads compiles to a branch that waits for each load in turn)
    const double *col = top ? Ta + kc : Tb + (kc - na);
    const int64_t ld = top ? lda : ldb;
    const int r0 = top ? 0 : na, rows = top ? na : nb;  // rows of this lane's triangle
#pragma unroll
    for (int j = 0; j < NP; j++) {
        const int jr = j - r0;
        r[j] = col[(int64_t)(jr < 0 ? 0 : (jr < rows ? jr : rows - 1)) * ld];
    }
#pragma unroll
    for (int j = 0; j < NP; j++) {
        const int jr = j - r0;
        r[j] = (col_ok && j <= k && jr >= 0 && jr < rows) ? r[j] : 0.0;
    }
    if (g.counts[CNT_G] > 0) {
        const double s2 = sqrt((double)g.m2[0]), s1 = sqrt((double)g.m1[0]);
        double h = k < na ? s2 * hA[k] : (col_ok ? s1 * hB[kc - na] : 0.0);
#pragma unroll
        for (int j = 0; j < NP; j++) {
            const double alpha = readlane_f64(r[j], j), hj = readlane_f64(h, j);
            const double q = fma(alpha, alpha, hj * hj);
            // (columns past the width hold zeros: hj = 0 leaves them alone)
            if (hj != 0.0 && q >= DBL_MIN) {
                const double rinv = rsq_refined(q);
                const double cs = alpha * rinv, sn = hj * rinv;
                if (k > j) {
                    const double a = r[j];
                    r[j] = fma(cs, a, sn * h);
                    h = fma(cs, h, -sn * a);
                } else if (k == j) {
                    r[j] = q * rinv;
                    h = 0.0;
                }
            }
        }
    }
    // row i: sign from its diagonal (lane i), or from its first nonzero entry if that is 0
#pragma unroll
    for (int i = 0; i < NP; i++) {
        if (i >= width) continue;
        const double d = readlane_f64(r[i], i);
        bool neg = d < 0.0;
        if (d == 0.0) {
            const unsigned long long nz = __ballot(col_ok && k >= i && r[i] != 0.0);
            if (nz) neg = readlane_f64(r[i], __builtin_ctzll(nz)) < 0.0;
        }
        if (col_ok) {
            const double v = k < i ? 0.0 : r[i];
            R[(int64_t)i * ldr + k] = (neg ? -v : v) + 0.0;
        }
    }
}

// One Cartesian root per workgroup: R in registers up to NP = 64, in LDS at NP = 128.
template <int NP>
__device__ __forceinline__ void merge_cartesian(const CartRoot &c)
{
    if constexpr (NP <= 64)
        merge_cartesian_reg<NP>(c.Ta, c.lda, c.na, c.Tb, c.ldb, c.nb, c.g, c.hA, c.hB, c.R, c.ldr);
    else
        merge_cartesian_lds<NP>(c.Ta, c.lda, c.na, c.Tb, c.ldb, c.nb, c.g, c.hA, c.hB, c.R, c.ldr);
}

template <int NP>
__global__ __launch_bounds__(64) void k_merge_cartesian(CartRoot c)
{
    merge_cartesian<NP>(c);
}

// A batch of Cartesian roots of one padded width (device table), one workgroup each.
template <int NP>
__global__ __launch_bounds__(64) void k_merge_cartesian_batch(const CartRoot *__restrict__ tab)
{
    const CartRoot c = tab[blockIdx.x];
    merge_cartesian<NP>(c);
}

hipError_t launch_merge_cartesian_batch(int np, const CartRoot *tab, int count, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    switch (np) {
#define FIGARO_MC(NPV) \
    case NPV: k_merge_cartesian_batch<NPV><<<(unsigned)count, 64, 0, s>>>(tab); return hipGetLastError();
    FIGARO_MC(4) FIGARO_MC(8) FIGARO_MC(16) FIGARO_MC(32) FIGARO_MC(64) FIGARO_MC(128)
#undef FIGARO_MC
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_merge_cartesian(int np, const double *Ta, int64_t lda, int na, const double *Tb, int64_t ldb, int nb,
                                  Groups g, const double *hA, const double *hB, double *R, int64_t ldr,
                                  hipStream_t s)
{
    if (na < 1 || nb < 1) return hipErrorInvalidValue;
    const CartRoot c{Ta, lda, na, Tb, ldb, nb, g, hA, hB, R, ldr};
    switch (np) {
#define FIGARO_MC(NPV) \
    case NPV: k_merge_cartesian<NPV><<<1, 64, 0, s>>>(c); return hipGetLastError();
    FIGARO_MC(4) FIGARO_MC(8) FIGARO_MC(16) FIGARO_MC(32) FIGARO_MC(64) FIGARO_MC(128)
#undef FIGARO_MC
    default: return hipErrorInvalidValue;
    }
}

__global__ void k_block_diag(const double *Ta, int64_t lda, int na, const double *Tb, int64_t ldb, int nb,
                             double *out, int64_t ldo)
{
    const int n = na + nb;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * ldo) return;
    const int i = (int)(e / ldo), k = (int)(e - (int64_t)i * ldo);
    double v = 0.0;
    if (i < na && k >= i && k < na) v = Ta[(int64_t)i * lda + k];
    else if (i >= na && k >= i && k < n) v = Tb[(int64_t)(i - na) * ldb + (k - na)];
    out[e] = v;
}

hipError_t launch_block_diag(const double *Ta, int64_t lda, int na, const double *Tb, int64_t ldb, int nb,
                             double *out, int64_t ldo, hipStream_t s)
{
    const int64_t total = (int64_t)(na + nb) * ldo;
    k_block_diag<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(Ta, lda, na, Tb, ldb, nb, out, ldo);
    return hipGetLastError();
}

hipError_t launch_sign_normalise(const void *Rin, int in_f64, int64_t ldin, int n, double *R,
                                 int64_t ldr, hipStream_t s)
{
    (void)in_f64;
    k_sign_normalise<<<n, 64, 0, s>>>((const double *)Rin, ldin, n, R, ldr);
    return hipGetLastError();
}

}  // namespace figaro
