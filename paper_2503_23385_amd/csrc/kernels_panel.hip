// Householder TSQR for wide rows streamed into a triangle: blocked (compact-WY)
// form of the structured update R <- triu(QR([R; X])) of the QR step
// (Experiments section; the stages of Section 1's reduction).  It reduces the
// regions of padded width 128 (a binary in-kernel tree over leaves) and merges
// triangles into roots of padded width up to 128 and the single head row of a
// wide Cartesian product; wider regions take the blocked QR of kernels_wqr.hip.
//
// One workgroup (4 waves) owns one triangle R, kept in FP64 in its output
// slot, and streams blocks of B rows X through LDS (B set by the LDS budget).
// For each panel of 16 columns [p0, p0 + 16):
//   1. panel factorisation: for each column j of the panel, the reflector of
//      [R_jj; X_:,j] (the same scalars as the narrow kernels: alpha = R_jj,
//      d_k = x_j . x_k, beta = -sign(alpha) sqrt(alpha^2 + d_j),
//      tau = 1 - alpha / beta, y_j = x_j / (alpha - beta)) is applied to the
//      panel's other columns; each wave owns B/4 rows and the dot products
//      are combined across waves through LDS (one barrier per column);
//   2. the panel's reflectors I - tau_j [e_j; y_j][e_j; y_j]^T are gathered
//      into the compact-WY form I - V T V^T with V = [I; Y]: the R part of
//      every v_j is a unit vector, so T follows from Y^T Y alone
//      (T_jj = tau_j, T_0:j,j = -tau_j T_0:j,0:j (Y^T Y)_0:j,j);
//   3. trailing update of columns c >= p0 + 16 in tiles of 16 columns
//      (one wave per tile): Z = R_p0:p0+16,c + Y^T X_:,c (MFMA), W = T^T Z,
//      R_p0:p0+16,c -= W, X_:,c -= Y W (MFMA).
// Reflector scalars, T and W are FP64; the products run in the storage type
// (FP64 MFMA for the plain form, FP32 MFMA for the mixed form).
#include <float.h>

#include "common.h"

namespace figaro {
namespace {

constexpr int kPanelThreads = 256;
constexpr int KB = 16;  // panel width (the MFMA tile)

template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
    typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct Vec4<double> {
    typedef double type __attribute__((ext_vector_type(4)));
};

// D (16 x 16) += A (16 x 4) B (4 x 16): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; element r of its result is D[drow(l / 16, r)][l % 16],
// with the row mapping of each instruction (measured on gfx950):
// FP32: 4 (l / 16) + r; FP64: (l / 16) + 4 r.
__device__ inline Vec4<float>::type mfma16(float a, float b, Vec4<float>::type c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline Vec4<double>::type mfma16(double a, double b, Vec4<double>::type c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename T>
__device__ inline int drow(int l4, int r)
{
    return sizeof(T) == 8 ? l4 + 4 * r : 4 * l4 + r;
}

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

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int64_t rows_of(const RowSrc &s) { return s.rows_dev ? *s.rows_dev : s.rows_host; }

template <int NP, typename Tacc>
struct PanelGeom {
    static constexpr int PAD = sizeof(Tacc) == 8 ? 2 : 4;
    static constexpr int LDX = NP + PAD;
    static constexpr int BUDGET = 136 * 1024;
    static constexpr int ROWB = LDX * (int)sizeof(Tacc);
    static constexpr int B = 256 * ROWB <= BUDGET ? 256
                           : 128 * ROWB <= BUDGET ? 128
                           : 64 * ROWB <= BUDGET  ? 64
                                                  : 32;
    static constexpr int RPW = B / 4;    // rows per wave
    static constexpr int RPL = RPW / 4;  // rows per lane in the panel step (4 row quarters per wave)
};

// LDS of one workgroup of the panel kernels.
template <int NP, typename Tacc>
struct PanelLds {
    using Gm = PanelGeom<NP, Tacc>;
    Tacc X[Gm::B * Gm::LDX];
    double Rpan[KB][KB + 1];  // the panel's diagonal block of R on entry (read only)
    double Rfin[KB][KB + 1];  // its rows once final (row j is final after column j)
    double red[2][4][KB];
    double tau[KB];
    double T[KB][KB + 1];
    double zb[4][KB][KB + 1];
    Tacc wb[4][KB][KB + 1];
    int flag;
};

// R (width rows x NP, FP64, global) <- init (or zero).
template <int NP>
__device__ inline void panel_set(double *R, const double *init, int64_t init_ld, int width)
{
    if (!init) {
        for (int e = threadIdx.x; e < width * NP; e += kPanelThreads) R[e] = 0.0;
        return;
    }
    staged_copy<8, double>(
        width * NP, threadIdx.x, kPanelThreads,
        [&](int e) {
            const int j = e / NP, k = e - j * NP;
            return init[(int64_t)j * init_ld + (k < width ? k : width - 1)];
        },
        [&](int e, double v) {
            const int j = e / NP, k = e - j * NP;
            R[e] = (k >= j && k < width) ? v : 0.0;
        });
}

// R absorbs rows [r_begin, r_end) of s0 then s1 (rows0 rows in s0), blocks of B rows.
template <int NP, typename Tin, typename Tacc>
__device__ void panel_absorb(PanelLds<NP, Tacc> &L, double *R, const RowSrc &s0, const RowSrc &s1, int64_t rows0,
                             int64_t r_begin, int64_t r_end, int tri_rows, int width)
{
    using Gm = PanelGeom<NP, Tacc>;
    using V4 = typename Vec4<Tacc>::type;
    constexpr int B = Gm::B, LDX = Gm::LDX, RPW = Gm::RPW, RPL = Gm::RPL;
    Tacc *X = L.X;
    auto &Rpan = L.Rpan;
    auto &Rfin = L.Rfin;
    auto &red = L.red;
    auto &tau = L.tau;
    auto &T = L.T;
    auto &zb = L.zb;
    auto &wb = L.wb;
    int par = 0;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int l16 = lane & 15, l4 = lane >> 4;
    for (int64_t rb = r_begin; rb < r_end; rb += B) {
        // rows past r_end read row r_end - 1 and are stored as zeros
        staged_copy<16, Tacc>(
            B * NP, tid, kPanelThreads,
            [&](int e) {
                const int i = e / NP, c = e - i * NP;
                const int64_t r = rb + i;
                return load_stacked<Tin, Tacc>(s0, s1, rows0, r < r_end ? r : r_end - 1, c);
            },
            [&](int e, Tacc v) {
                const int i = e / NP, c = e - i * NP;
                const int64_t r = rb + i;
                const bool real = r < r_end && c < width && stacked_real(s0, s1, rows0, r, c);
                X[i * LDX + c] = real ? v : Tacc(0);
            });
        // Leading columns known to be zero in this block.
        int jstart = 0;
        const int64_t rlast = min(r_end, rb + B) - 1;
        if (rlast < rows0) jstart = s0.col_off;
        else if (rb >= rows0) jstart = s1.col_off;
        if (tri_rows > 0 && (rlast < rows0 || rb >= rows0)) {
            const int64_t lr = rb < rows0 ? rb : rb - rows0;
            const int64_t off = lr % tri_rows;
            if (off + B <= tri_rows) jstart += (int)off;
        }
        __syncthreads();

        for (int p0 = (jstart / KB) * KB; p0 < width; p0 += KB) {
            const int kb = min(KB, width - p0);
            {
                const int i = tid / KB, k = tid % KB;
                Rpan[i][k] = (i < kb && k < kb && k >= i) ? R[(int64_t)(p0 + i) * NP + p0 + k] : 0.0;
                if (tid < KB) tau[tid] = 0.0;
            }
            __syncthreads();

            // ---- 1. panel factorisation
            Tacc *xr = X + (wv * RPW + l4 * RPL) * LDX + p0;
            for (int j = 0; j < kb; j++) {
                double d = 0.0;
#pragma unroll
                for (int i = 0; i < RPL; i++) d = fma((double)xr[i * LDX + j], (double)xr[i * LDX + l16], d);
                d += __shfl_xor(d, 16, 64);
                d += __shfl_xor(d, 32, 64);
                if (l4 == 0) red[par][wv][l16] = d;
                __syncthreads();
                const double dk = ((red[par][0][l16] + red[par][1][l16]) + red[par][2][l16]) + red[par][3][l16];
                const double s = ((red[par][0][j] + red[par][1][j]) + red[par][2][j]) + red[par][3][j];
                par ^= 1;
                const double alpha = Rpan[j][j];
                const double q = fma(alpha, alpha, s);
                double tj = 0.0, beta = alpha, scl = 0.0, inv_beta = 0.0;
                if (s > 0.0 && q >= DBL_MIN) {
                    const double r = rsq_refined(q);
                    const double sg = alpha >= 0.0 ? 1.0 : -1.0;
                    const double nrm = q * r;
                    beta = -sg * nrm;
                    inv_beta = -sg * r;
                    scl = rcp_refined(alpha + sg * nrm);
                    tj = 1.0 - alpha * inv_beta;
                }
                // Row j of R changes only here: the new values go to Rfin, so Rpan stays
                // valid for the waves still reading it in this step.
                const double rjk = Rpan[j][l16];
                double rnew = rjk;
                if (tj != 0.0 && l16 > j && l16 < kb) {
                    const double w = rjk + scl * dk;
                    const Tacc c = (Tacc)(w * inv_beta);
#pragma unroll
                    for (int i = 0; i < RPL; i++) xr[i * LDX + l16] += c * xr[i * LDX + j];
                    rnew = rjk - tj * w;
                }
                if (l16 == j && tj != 0.0) rnew = beta;
                if (wv == 0 && l4 == 0) Rfin[j][l16] = rnew;
                wave_sync();
                if (l16 == j) {
#pragma unroll
                    for (int i = 0; i < RPL; i++) xr[i * LDX + j] = (Tacc)((double)xr[i * LDX + j] * scl);
                }
                if (tid == 0) tau[j] = tj;
                wave_sync();
            }
            __syncthreads();
            {
                const int i = tid / KB, k = tid % KB;
                if (i < kb && k < kb && k >= i) R[(int64_t)(p0 + i) * NP + p0 + k] = Rfin[i][k];
            }

            // ---- 2. T from Y^T Y (per-wave partial Gram on MFMA, summed in a fixed order)
            {
                V4 acc = {0, 0, 0, 0};
#pragma unroll 4
                for (int kk = 0; kk < RPW / 4; kk++) {
                    const Tacc a = X[(wv * RPW + 4 * kk + l4) * LDX + p0 + l16];
                    acc = mfma16(a, a, acc);
                }
#pragma unroll
                for (int r = 0; r < 4; r++) zb[wv][drow<Tacc>(l4, r)][l16] = (double)acc[r];
            }
            __syncthreads();
            if (wv == 0) {
                for (int e = lane; e < KB * KB; e += 64) {
                    const int i = e / KB, k = e % KB;
                    zb[0][i][k] = ((zb[0][i][k] + zb[1][i][k]) + zb[2][i][k]) + zb[3][i][k];
                }
                wave_sync();
                if (lane < KB) {
                    // row i = lane of T: T_ii = tau_i, T_ij = -tau_j sum_{k=i}^{j-1} T_ik G_kj
                    const int i = lane;
                    double trow[KB];
#pragma unroll
                    for (int j = 0; j < KB; j++) trow[j] = 0.0;
                    trow[i] = tau[i];
#pragma unroll
                    for (int j = 0; j < KB; j++) {
                        if (j > i) {
                            double acc = 0.0;
#pragma unroll
                            for (int k = 0; k < KB; k++)
                                if (k >= i && k < j) acc = fma(trow[k], zb[0][k][j], acc);
                            trow[j] = -tau[j] * acc;
                        }
                    }
#pragma unroll
                    for (int j = 0; j < KB; j++) T[i][j] = trow[j];
                }
            }
            __syncthreads();

            // ---- 3. trailing update, one wave per 16-column tile
            for (int c0 = p0 + KB + wv * KB; c0 < width; c0 += 4 * KB) {
                const int n = c0 + l16;
                double rold[4];
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int m = drow<Tacc>(l4, r);
                    rold[r] = (m < kb && n < width) ? R[(int64_t)(p0 + m) * NP + n] : 0.0;
                }
                V4 acc = {0, 0, 0, 0};
#pragma unroll 8
                for (int kk = 0; kk < B / 4; kk++) {
                    const int row = 4 * kk + l4;
                    acc = mfma16(X[row * LDX + p0 + l16], X[row * LDX + c0 + l16], acc);
                }
#pragma unroll
                for (int r = 0; r < 4; r++) zb[wv][drow<Tacc>(l4, r)][l16] = rold[r] + (double)acc[r];
                wave_sync();
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int m = drow<Tacc>(l4, r);
                    double w = 0.0;
                    for (int k = 0; k <= m; k++) w = fma(T[k][m], zb[wv][k][l16], w);
                    if (m < kb && n < width) R[(int64_t)(p0 + m) * NP + n] = rold[r] - w;
                    wb[wv][m][l16] = (Tacc)w;
                }
                wave_sync();
                for (int rt = 0; rt < B / 16; rt++) {
                    V4 dd = {0, 0, 0, 0};
#pragma unroll
                    for (int kk = 0; kk < 4; kk++)
                        dd = mfma16(X[(rt * 16 + l16) * LDX + p0 + 4 * kk + l4], wb[wv][4 * kk + l4][l16], dd);
#pragma unroll
                    for (int r = 0; r < 4; r++) X[(rt * 16 + drow<Tacc>(l4, r)) * LDX + c0 + l16] -= dd[r];
                }
                wave_sync();
            }
            __syncthreads();
        }
    }
}

template <int NP, typename Tin, typename Tacc>
__global__ __launch_bounds__(kPanelThreads) void k_tsqr_panel(const double *init, int64_t init_ld, RowSrc s0,
                                                              RowSrc s1, int nsrc, int width, int tri_rows,
                                                              double *tri_out, int64_t tri_stride)
{
    __shared__ PanelLds<NP, Tacc> L;
    static_assert(sizeof(PanelLds<NP, Tacc>) <= 160 * 1024, "LDS budget");
    double *R = tri_out + (int64_t)blockIdx.x * tri_stride;  // width rows x NP
    panel_set<NP>(R, init, init_ld, width);
    const int64_t rows0 = rows_of(s0);
    const int64_t total = rows0 + (nsrc > 1 ? rows_of(s1) : 0);
    int64_t chunk = (total + gridDim.x - 1) / gridDim.x;
    chunk = ((chunk + PanelGeom<NP, Tacc>::B - 1) / PanelGeom<NP, Tacc>::B) * PanelGeom<NP, Tacc>::B;
    const int64_t r_begin = (int64_t)blockIdx.x * chunk;
    const int64_t r_end = min(total, r_begin + chunk);
    __syncthreads();
    panel_absorb<NP, Tin, Tacc>(L, R, s0, s1, rows0, r_begin, r_end, tri_rows, width);
}

// Up to two regions of the same padded width in one launch, each reduced by an in-kernel
// binary tree.  The number of leaves follows the region's row count on the device:
// min(nleaves, ceil(rows / rows_per_leaf)); the remaining workgroups leave at once.
// Leaf g reduces its rows into slot g of level 0; at each node the last child to arrive
// (per-node atomic counter) writes the parent: the first child's triangle absorbing the
// second's.  A lone child is copied up.  The last level's triangle is copied to root.
template <int NP, typename Tin, typename Tacc>
__global__ __launch_bounds__(kPanelThreads) void k_tsqr_panel_tree(TreeRegion reg0, TreeRegion reg1)
{
    __shared__ PanelLds<NP, Tacc> L;
    static_assert(sizeof(PanelLds<NP, Tacc>) <= 160 * 1024, "LDS budget");
    constexpr int B = PanelGeom<NP, Tacc>::B;
    int g = blockIdx.x;
    const bool second = g >= reg0.nleaves;
    const TreeRegion rg = second ? reg1 : reg0;
    if (second) g -= reg0.nleaves;
    const int width = rg.width;
    const int64_t rows = rows_of(rg.src);
    const int64_t want = (rows + rg.rows_per_leaf - 1) / rg.rows_per_leaf;
    const int nleaves = (int)max((int64_t)1, min((int64_t)rg.nleaves, want));
    if (g >= nleaves) return;
    const int64_t tsz = (int64_t)width * NP;
    int64_t chunk = (rows + nleaves - 1) / nleaves;
    chunk = ((chunk + B - 1) / B) * B;
    const int64_t r_begin = (int64_t)g * chunk, r_end = min(rows, r_begin + chunk);
    double *R = rg.slots + (int64_t)g * tsz;
    panel_set<NP>(R, nullptr, 0, width);
    __syncthreads();
    const RowSrc none{};
    panel_absorb<NP, Tin, Tacc>(L, R, rg.src, none, rows, r_begin, r_end, 0, width);

    int node = g, n = nleaves;
    int64_t soff = 0, coff = 0;
    while (n > 1) {
        const int parent = node >> 1, first = parent << 1;
        const int nchild = min(2, n - first);
        double *P = rg.slots + (soff + n + parent) * tsz;
        if (nchild > 1) {
            __syncthreads();
            if (threadIdx.x == 0) {
                __threadfence();
                L.flag = __hip_atomic_fetch_add(&rg.counters[coff + parent], 1, __ATOMIC_ACQ_REL,
                                                __HIP_MEMORY_SCOPE_AGENT);
                __threadfence();
            }
            __syncthreads();
            if (L.flag != 1) return;  // the last child to arrive combines this node
            panel_set<NP>(P, rg.slots + (soff + first) * tsz, NP, width);
            __syncthreads();
            const RowSrc sib{rg.slots + (soff + first + 1) * tsz, nullptr, width, NP, 0, width};
            panel_absorb<NP, double, Tacc>(L, P, sib, none, width, 0, width, width, width);
        } else {
            __syncthreads();
            for (int e = threadIdx.x; e < tsz; e += kPanelThreads) P[e] = R[e];
        }
        R = P;
        node = parent;
        soff += n;
        coff += (n + 1) / 2;
        n = (n + 1) / 2;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < tsz; e += kPanelThreads) rg.root[e] = R[e];
}

template <int NP>
hipError_t launch_panel_np(int acc_f64, int in_f64, const double *init, int64_t init_ld, RowSrc s0, RowSrc s1,
                           int nsrc, int width, int tri_rows, int nwg, double *tri, int64_t stride, hipStream_t s)
{
#define FIGARO_PANEL(TI, TA) \
    k_tsqr_panel<NP, TI, TA><<<nwg, kPanelThreads, 0, s>>>(init, init_ld, s0, s1, nsrc, width, tri_rows, tri, stride)
    if (acc_f64) {
        if (in_f64) FIGARO_PANEL(double, double);
        else FIGARO_PANEL(float, double);
    } else {
        if (in_f64) FIGARO_PANEL(double, float);
        else FIGARO_PANEL(float, float);
    }
#undef FIGARO_PANEL
    return hipGetLastError();
}

template <int NP>
hipError_t launch_panel_tree_np(int acc_f64, int in_f64, const TreeRegion *regs, int nreg, hipStream_t s)
{
    TreeRegion r0 = regs[0];
    TreeRegion r1 = nreg > 1 ? regs[1] : TreeRegion{};
    const unsigned grid = (unsigned)(r0.nleaves + r1.nleaves);
#define FIGARO_PTREE(TI, TA) k_tsqr_panel_tree<NP, TI, TA><<<grid, kPanelThreads, 0, s>>>(r0, r1)
    if (acc_f64) {
        if (in_f64) FIGARO_PTREE(double, double);
        else FIGARO_PTREE(float, double);
    } else {
        if (in_f64) FIGARO_PTREE(double, float);
        else FIGARO_PTREE(float, float);
    }
#undef FIGARO_PTREE
    return hipGetLastError();
}

}  // namespace

hipError_t launch_tsqr_panel_tree(int np, int acc_f64, int in_f64, const TreeRegion *regs, int nreg, hipStream_t s)
{
    if (nreg < 1 || nreg > 2) return hipErrorInvalidValue;
    switch (np) {
    case 128: return launch_panel_tree_np<128>(acc_f64, in_f64, regs, nreg, s);
    case 256: return launch_panel_tree_np<256>(acc_f64, in_f64, regs, nreg, s);
    case 512: return launch_panel_tree_np<512>(acc_f64, in_f64, regs, nreg, s);
    default: return hipErrorInvalidValue;
    }
}

void tsqr_panel_tree_sizes(int nleaves, int64_t *slots, int64_t *counters)
{
    int64_t sl = 0, c = 0;
    int n = nleaves;
    while (n > 1) {
        sl += n;
        c += (n + 1) / 2;
        n = (n + 1) / 2;
    }
    *slots = sl + 1;  // every level's nodes plus the last level's single node
    *counters = c + 1;
}

int tsqr_panel_rows(int np, int acc_f64)
{
    switch (np) {
    case 128: return acc_f64 ? PanelGeom<128, double>::B : PanelGeom<128, float>::B;
    case 256: return acc_f64 ? PanelGeom<256, double>::B : PanelGeom<256, float>::B;
    case 512: return acc_f64 ? PanelGeom<512, double>::B : PanelGeom<512, float>::B;
    default: return 0;
    }
}

hipError_t launch_tsqr_panel(int np, int acc_f64, int in_f64, const double *init, int64_t init_ld, RowSrc s0,
                             RowSrc s1, int nsrc, int width, int tri_rows, int nwg, double *tri, int64_t tri_stride,
                             hipStream_t s)
{
    if (nwg < 1 || width < 1 || width > np) return hipErrorInvalidValue;
    switch (np) {
    case 128: return launch_panel_np<128>(acc_f64, in_f64, init, init_ld, s0, s1, nsrc, width, tri_rows, nwg, tri, tri_stride, s);
    case 256: return launch_panel_np<256>(acc_f64, in_f64, init, init_ld, s0, s1, nsrc, width, tri_rows, nwg, tri, tri_stride, s);
    case 512: return launch_panel_np<512>(acc_f64, in_f64, init, init_ld, s0, s1, nsrc, width, tri_rows, nwg, tri, tri_stride, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace figaro
