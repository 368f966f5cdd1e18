// Householder TSQR for wide rows (padded widths 128, 256, 512): every leaf's rows are
// factorised at once by the blocked (compact-WY) Householder QR, panel by panel, and the
// leaves' triangles are merged pairwise up a binary in-kernel tree; the QR step of the
// compact matrix (Experiments section; the reduction of Section 1).  One workgroup of
// 512 threads per leaf; the rows stay in global memory (in place) and only a panel's
// 16 columns are held in registers.
//
// A problem is a set of rows of width w, the "active rows" of panel [p0, p0 + 16):
//   leaf:  rows [p0, m) of the leaf (storage type S: the compact matrix's type);
//   merge: rows [p0, p0 + 16) of a top triangle and rows [0, p0 + 16) of a bottom one
//          (FP64 node triangles; the bottom triangle's later rows are zero in every
//          column >= p0 and stay zero).
// Per panel:
//   1. column steps with the reflector scalars of the narrow kernels (alpha = pivot,
//      d_k = x_j . x_k over the rows below it, beta = -sign(alpha) sqrt(alpha^2 + d_j),
//      tau = 1 - alpha / beta, v = x_j / (alpha - beta)).  Thread (k, g) holds column
//      p0 + k of active rows g, g + 32, ... in registers; the pivot column goes through
//      LDS, the dot products are reduced over the 32 row groups (two shuffles inside a
//      wave, then the 8 wave partials summed in a fixed order);
//   2. the reflectors leave the matrix: V (unit lower trapezoidal, with its 1s and 0s
//      written out) goes to a side buffer, the panel's columns keep R on and above the
//      diagonal and zeros below;
//   3. trailing update of the columns right of the panel in 16-column subtiles (up to
//      four per wave): Z = V^T A and G = V^T V on the matrix cores (V staged through LDS
//      in chunks of 256 rows), T from G and tau (T_ii = tau_i,
//      T_ij = -tau_j sum_{k=i..j-1} T_ik G_kj), W = T^T Z, A -= V W on the matrix cores.
// Products run in the storage type (FP32 or FP64 matrix cores), reflector scalars, T
// and W in FP64; merges are FP64 throughout.
#include <float.h>

#include "common.h"

namespace figaro {
namespace {

constexpr int kQb = 16;                     // panel width (the MFMA tile)
constexpr int kQThreads = 512;              // 8 waves, two per SIMD (256 registers each)
constexpr int kQWaves = kQThreads / 64;
constexpr int kQGroups = kQThreads / kQb;   // 32 row groups of the column steps
constexpr int kQCh = 256;                   // rows of V staged per chunk of the update
constexpr int kQSub = 32 / kQWaves;         // 16-column subtiles per wave (at most 31 + G)

constexpr int kQMergeRpt = (kQb + 512 + kQGroups - 1) / kQGroups;  // rows per thread of a merge

template <typename S>
struct QGeom {
    static constexpr int RPT = 32;                        // active rows per thread
    static constexpr int MAXR = kQGroups * RPT;           // active rows of a problem
};

// Bytes of one workgroup's reflector side buffer: V of a leaf panel (MAXR x 16 of the
// storage type) or of a merge panel (up to 16 + 512 rows x 16 FP64).
constexpr int64_t kQVbufBytes = (int64_t)kQb * (kQGroups * QGeom<double>::RPT * (int64_t)sizeof(double) >
                                                        (kQb + 512) * (int64_t)sizeof(double)
                                                    ? kQGroups * QGeom<double>::RPT * (int64_t)sizeof(double)
                                                    : (kQb + 512) * (int64_t)sizeof(double));
static_assert(kQVbufBytes >= (int64_t)kQb * QGeom<float>::MAXR * (int64_t)sizeof(float), "side buffer");

template <typename T>
struct QVec4;
template <>
struct QVec4<float> {
    typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct QVec4<double> {
    typedef double type __attribute__((ext_vector_type(4)));
};

// D (16 x 16) += A (16 x 4) B (4 x 16): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; element r of its result is D[qrow_of(l / 16, r)][l % 16]
// (FP32: 4 (l / 16) + r; FP64: (l / 16) + 4 r, measured on gfx950).
__device__ inline QVec4<float>::type qmfma(float a, float b, QVec4<float>::type c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline QVec4<double>::type qmfma(double a, double b, QVec4<double>::type c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <typename S>
__device__ inline int qrow_of(int l4, int r)
{
    return sizeof(S) == 8 ? l4 + 4 * r : 4 * l4 + r;
}

__device__ inline double q_rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    r = fma(fma(-x, r, 1.0), r, r);
    return r;
}
__device__ inline double q_rsq(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * fma(-hx * y, y, 1.5);
    y = y * fma(-hx * y, y, 1.5);
    return y;
}

__device__ inline void q_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Buffer-resource access (descriptor word 3 of a raw 32-bit buffer on gfx9-family GPUs):
// one 32-bit offset per access, and an access at an offset past the buffer's size reads
// 0 and writes nothing.
constexpr int kQWord3 = 0x00020000;
constexpr uint32_t kQOob = 0x80000000u;  // past every buffer here (all below 2^31 bytes)

template <typename S>
__device__ inline S qld(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ inline float qld<float>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
template <>
__device__ inline double qld<double>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ inline void qst(__amdgpu_buffer_rsrc_t r, uint32_t off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, 0);
}
__device__ inline void qst(__amdgpu_buffer_rsrc_t r, uint32_t off, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r,
                                          (int)off, 0, 0);
}

// The active rows of one panel as two byte ranges: rows [0, n0) in range 0 (stride ld0
// bytes), rows [n0, n0 + n1) in range 1 (stride ld1); columns [0, w).  An access outside
// them (row past the active rows, column >= w) reads 0 and writes nothing.
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

template <typename S>
struct QBuf {
    __amdgpu_buffer_rsrc_t r0, r1;
    uint32_t ld0, ld1;
    int n0, n1, w;
    __device__ uint32_t off0(int a, int c) const
    {
        return (a < n0 && c < w) ? (uint32_t)a * ld0 + (uint32_t)c * (uint32_t)sizeof(S) : kQOob;
    }
    __device__ uint32_t off1(int a, int c) const
    {
        return (a >= n0 && a < n0 + n1 && c < w) ? (uint32_t)(a - n0) * ld1 + (uint32_t)c * (uint32_t)sizeof(S)
                                                 : kQOob;
    }
    __device__ S load(int a, int c) const
    {
        S v = qld<S>(r0, off0(a, c));
        if (n1 > 0) v += qld<S>(r1, off1(a, c));  // one of the two reads is 0
        return v;
    }
    __device__ void store(int a, int c, S v) const
    {
        qst(r0, off0(a, c), v);
        if (n1 > 0) qst(r1, off1(a, c), v);
    }
    // 16 bytes at (row a, columns [c, c + 16 / sizeof(S))): callers keep c + that <= w
    __device__ u32x4 load16(int a, int c) const
    {
        u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r0, (int)off0(a, c), 0, 0);
        if (n1 > 0) {
            const u32x4 v1 = __builtin_amdgcn_raw_buffer_load_b128(r1, (int)off1(a, c), 0, 0);
            v |= v1;  // one of the two reads is all zero bits
        }
        return v;
    }
    __device__ void store16(int a, int c, u32x4 v) const
    {
        __builtin_amdgcn_raw_buffer_store_b128(v, r0, (int)off0(a, c), 0, 0);
        if (n1 > 0) __builtin_amdgcn_raw_buffer_store_b128(v, r1, (int)off1(a, c), 0, 0);
    }
};

template <typename S>
__device__ inline QBuf<S> qbuf(S *b0, int64_t ld0, int n0, S *b1, int64_t ld1, int n1, int w)
{
    QBuf<S> q;
    const int64_t e = (int64_t)sizeof(S);
    q.r0 = __builtin_amdgcn_make_buffer_rsrc(b0, (short)0, (int)(n0 * ld0 * e), kQWord3);
    q.r1 = __builtin_amdgcn_make_buffer_rsrc(n1 > 0 ? b1 : b0, (short)0, n1 > 0 ? (int)(n1 * ld1 * e) : 0, kQWord3);
    q.ld0 = (uint32_t)(ld0 * e);
    q.ld1 = (uint32_t)(ld1 * e);
    q.n0 = n0;
    q.n1 = n1;
    q.w = w;
    return q;
}

// A value the whole wave holds (read from lane 0), so that the compiler keeps it, and what
// is derived from it (buffer descriptors above all), in scalar registers.
__device__ inline int64_t q_uniform(int64_t v)
{
    const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

template <typename S>
struct QLds {
    union {
        struct {
            S col[2][QGeom<S>::MAXR];  // the pivot column of a step, row group major
            double red[2][kQWaves][kQb];
            double piv[2][kQb];
        } f;
        struct {
            S vch[kQCh][kQb + 1];
            double zb[kQWaves][kQb][kQb + 1];
            S wb[kQWaves][kQSub][kQb][kQb + 1];
            double G[kQb][kQb + 1];
            double T[kQb][kQb + 1];
        } u;
    };
    double tau[kQb];
    int flag;
};

// T of the panel (wave 0, lanes 0..15 own a row each, left to right in LDS) from
// G = V^T V in LDS and the panel's tau.
template <typename S>
__device__ inline void q_make_t(QLds<S> &L, int wv, int lane)
{
    if (wv == 0 && lane < kQb) {
        const int i = lane;
        for (int jj = 0; jj < kQb; jj++) L.u.T[i][jj] = jj == i ? L.tau[i] : 0.0;
        for (int jj = i + 1; jj < kQb; jj++) {
            double a = 0.0;
            for (int kk = i; kk < jj; kk++) a = fma(L.u.T[i][kk], L.u.G[kk][jj], a);
            L.u.T[i][jj] = -L.tau[jj] * a;
        }
    }
}

// V chunk [rb, rb + kQCh) of the side buffer into LDS (rows past na as zeros).
template <typename S>
__device__ inline void q_stage_v(QLds<S> &L, const S *vbuf, int rb, int na)
{
    for (int e = threadIdx.x; e < kQCh * kQb; e += kQThreads) {
        const int rr = e / kQb, kk = e % kQb;
        L.u.vch[rr][kk] = rb + rr < na ? vbuf[(int64_t)(rb + rr) * kQb + kk] : S(0);
    }
}

// Trailing update, one 16-column subtile per access (any width).
template <typename S>
__device__ void q_trail_scalar(QLds<S> &L, const QBuf<S> &q, const S *vbuf, int na, int c0, int width, int wv,
                               int lane)
{
    using V4 = typename QVec4<S>::type;
    const int l16 = lane & 15, l4 = lane >> 4;
        const int nsub = (width - c0 + kQb - 1) / kQb;  // subtile nsub is G = V^T V
        V4 acc[kQSub];
#pragma unroll
        for (int u = 0; u < kQSub; u++) acc[u] = V4{0, 0, 0, 0};
        for (int rb = 0; rb < na; rb += kQCh) {
            q_stage_v<S>(L, vbuf, rb, na);
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kQSub; u++) {
                const int s = wv + kQWaves * u;
                if (s > nsub) continue;
                if (s == nsub) {
                    const int nk = min(kQCh, na - rb + 3) / 4;
                    for (int kk = 0; kk < nk; kk++) {
                        const S a = L.u.vch[4 * kk + l4][l16];
                        acc[u] = qmfma(a, a, acc[u]);
                    }
                } else {
                    const int col = c0 + kQb * s + l16;
                    // batches of 16 loads, the next batch in flight during a batch's products
                    // (rows past the active ones read 0, and whole batches past them are skipped)
                    const int nk = min(kQCh, na - rb + 3) / 4;
                    constexpr int NB = 8;
                    S b[NB], bn[NB];
#pragma unroll
                    for (int kk = 0; kk < NB; kk++) b[kk] = q.load(rb + 4 * kk + l4, col);
                    for (int k0 = 0; k0 < nk; k0 += NB) {
                        if (k0 + NB < nk) {
#pragma unroll
                            for (int kk = 0; kk < NB; kk++) bn[kk] = q.load(rb + 4 * (k0 + NB + kk) + l4, col);
                        }
#pragma unroll
                        for (int kk = 0; kk < NB; kk++)
                            acc[u] = qmfma(L.u.vch[4 * (k0 + kk) + l4][l16], b[kk], acc[u]);
#pragma unroll
                        for (int kk = 0; kk < NB; kk++) b[kk] = bn[kk];
                    }
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int u = 0; u < kQSub; u++) {
            if (wv + kQWaves * u == nsub) {
#pragma unroll
                for (int r = 0; r < 4; r++) L.u.G[qrow_of<S>(l4, r)][l16] = (double)acc[u][r];
            }
        }
        __syncthreads();
        q_make_t<S>(L, wv, lane);
        __syncthreads();
        // W = T^T Z for each of the wave's subtiles
#pragma unroll
        for (int u = 0; u < kQSub; u++) {
            if (wv + kQWaves * u >= nsub) continue;
#pragma unroll
            for (int r = 0; r < 4; r++) L.u.zb[wv][qrow_of<S>(l4, r)][l16] = (double)acc[u][r];
            q_wave_sync();
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int mm = qrow_of<S>(l4, r);
                double w = 0.0;
                for (int kk = 0; kk <= mm; kk++) w = fma(L.u.T[kk][mm], L.u.zb[wv][kk][l16], w);
                L.u.wb[wv][u][mm][l16] = (S)w;
            }
            q_wave_sync();
        }
        // A -= V W
        for (int rb = 0; rb < na; rb += kQCh) {
            __syncthreads();
            q_stage_v<S>(L, vbuf, rb, na);
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kQSub; u++) {
                const int s = wv + kQWaves * u;
                if (s >= nsub) continue;
                const int col = c0 + kQb * s + l16;
                // two 16-row blocks at a time: their 8 loads first, then products and stores
                for (int sub0 = 0; sub0 < kQCh / 16; sub0 += 2) {
                    if (rb + 16 * sub0 >= na) break;
                    S cur[2][4];
#pragma unroll
                    for (int b4 = 0; b4 < 2; b4++)
#pragma unroll
                        for (int r = 0; r < 4; r++)
                            cur[b4][r] = q.load(rb + 16 * (sub0 + b4) + qrow_of<S>(l4, r), col);
#pragma unroll
                    for (int b4 = 0; b4 < 2; b4++) {
                        V4 d = {0, 0, 0, 0};
#pragma unroll
                        for (int kk = 0; kk < 4; kk++)
                            d = qmfma(L.u.vch[16 * (sub0 + b4) + l16][4 * kk + l4], L.u.wb[wv][u][4 * kk + l4][l16],
                                      d);
#pragma unroll
                        for (int r = 0; r < 4; r++)
                            q.store(rb + 16 * (sub0 + b4) + qrow_of<S>(l4, r), col, cur[b4][r] - d[r]);
                    }
                }
            }
        }
}

// Trailing update with 16-byte accesses (width a multiple of VW = 16 / sizeof(S)): wave
// wv owns groups gi = wv, wv + 8, ... of 16 VW columns; within a group, subtile v holds
// columns c0 + 16 VW gi + VW n + v (n = 0..15), so that a lane's 16 bytes at columns
// VW l16 .. VW l16 + VW - 1 of the group are column l16 of subtiles 0..VW-1.
// The last wave also forms G = V^T V.
template <typename S>
__device__ void q_trail_vec(QLds<S> &L, const QBuf<S> &q, const S *vbuf, int na, int c0, int width, int wv,
                            int lane)
{
    using V4 = typename QVec4<S>::type;
    constexpr int VW = 16 / (int)sizeof(S);
    constexpr int GPW = kQSub / VW;  // groups per wave
    typedef S SV __attribute__((ext_vector_type(VW)));
    const int l16 = lane & 15, l4 = lane >> 4;
    const int ng = (width - c0 + 16 * VW - 1) / (16 * VW);
    const bool gwave = wv == kQWaves - 1;
    V4 acc[GPW][VW], accg = {0, 0, 0, 0};
#pragma unroll
    for (int u = 0; u < GPW; u++)
#pragma unroll
        for (int v = 0; v < VW; v++) acc[u][v] = V4{0, 0, 0, 0};
    for (int rb = 0; rb < na; rb += kQCh) {
        q_stage_v<S>(L, vbuf, rb, na);
        __syncthreads();
        const int nk = min(kQCh, na - rb + 3) / 4;
#pragma unroll
        for (int u = 0; u < GPW; u++) {
            const int gi = wv + kQWaves * u;
            if (gi >= ng) continue;
            const int col = c0 + 16 * VW * gi + VW * l16;  // past the width: reads 0
            constexpr int NB = 8;
            u32x4 b[NB], bn[NB];
#pragma unroll
            for (int kk = 0; kk < NB; kk++) b[kk] = q.load16(rb + 4 * kk + l4, col);
            for (int k0 = 0; k0 < nk; k0 += NB) {
                if (k0 + NB < nk) {
#pragma unroll
                    for (int kk = 0; kk < NB; kk++) bn[kk] = q.load16(rb + 4 * (k0 + NB + kk) + l4, col);
                }
#pragma unroll
                for (int kk = 0; kk < NB; kk++) {
                    const S a = L.u.vch[4 * (k0 + kk) + l4][l16];
                    const SV bv = __builtin_bit_cast(SV, b[kk]);
#pragma unroll
                    for (int v = 0; v < VW; v++) acc[u][v] = qmfma(a, bv[v], acc[u][v]);
                }
#pragma unroll
                for (int kk = 0; kk < NB; kk++) b[kk] = bn[kk];
            }
        }
        if (gwave) {
            for (int kk = 0; kk < nk; kk++) {
                const S a = L.u.vch[4 * kk + l4][l16];
                accg = qmfma(a, a, accg);
            }
        }
        __syncthreads();
    }
    if (gwave) {
#pragma unroll
        for (int r = 0; r < 4; r++) L.u.G[qrow_of<S>(l4, r)][l16] = (double)accg[r];
    }
    __syncthreads();
    q_make_t<S>(L, wv, lane);
    __syncthreads();
    // W = T^T Z for each subtile of the wave's groups (wb slot VW u + v)
#pragma unroll
    for (int u = 0; u < GPW; u++) {
        if (wv + kQWaves * u >= ng) continue;
#pragma unroll
        for (int v = 0; v < VW; v++) {
#pragma unroll
            for (int r = 0; r < 4; r++) L.u.zb[wv][qrow_of<S>(l4, r)][l16] = (double)acc[u][v][r];
            q_wave_sync();
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int mm = qrow_of<S>(l4, r);
                double w = 0.0;
                for (int kk = 0; kk <= mm; kk++) w = fma(L.u.T[kk][mm], L.u.zb[wv][kk][l16], w);
                L.u.wb[wv][VW * u + v][mm][l16] = (S)w;
            }
            q_wave_sync();
        }
    }
    // A -= V W, two 16-row blocks at a time: their loads first, then products and stores
    for (int rb = 0; rb < na; rb += kQCh) {
        __syncthreads();
        q_stage_v<S>(L, vbuf, rb, na);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < GPW; u++) {
            const int gi = wv + kQWaves * u;
            if (gi >= ng) continue;
            const int col = c0 + 16 * VW * gi + VW * l16;
            for (int sub0 = 0; sub0 < kQCh / 16; sub0 += 2) {
                if (rb + 16 * sub0 >= na) break;
                u32x4 cur[2][4];
#pragma unroll
                for (int b4 = 0; b4 < 2; b4++)
#pragma unroll
                    for (int r = 0; r < 4; r++) cur[b4][r] = q.load16(rb + 16 * (sub0 + b4) + qrow_of<S>(l4, r), col);
#pragma unroll
                for (int b4 = 0; b4 < 2; b4++) {
                    V4 d[VW];
#pragma unroll
                    for (int v = 0; v < VW; v++) {
                        d[v] = V4{0, 0, 0, 0};
#pragma unroll
                        for (int kk = 0; kk < 4; kk++)
                            d[v] = qmfma(L.u.vch[16 * (sub0 + b4) + l16][4 * kk + l4],
                                         L.u.wb[wv][VW * u + v][4 * kk + l4][l16], d[v]);
                    }
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        SV x = __builtin_bit_cast(SV, cur[b4][r]);
#pragma unroll
                        for (int v = 0; v < VW; v++) x[v] -= d[v][r];
                        q.store16(rb + 16 * (sub0 + b4) + qrow_of<S>(l4, r), col, __builtin_bit_cast(u32x4, x));
                    }
                }
            }
        }
    }
}

// Blocked QR of one problem in place.  kind 0 (leaf): rows [0, m) at X (stride ld);
// kind 1 (merge): top triangle X (stride ld), bottom triangle Y (stride ldy), width rows
// each.  vbuf holds V of the current panel (MAXR x 16).
// RPT: active rows per thread (a leaf up to MAXR rows in all; a merge at most 16 + 512,
// 17 per row group).
template <typename S, int RPT>
__device__ __forceinline__ void q_factor(QLds<S> &L, int kind, S *X, int64_t ld, int64_t m, S *Y, int64_t ldy, int width, S *vbuf)
{
    static_assert(kQGroups * RPT <= QGeom<S>::MAXR, "pivot column buffer");
    const int t = threadIdx.x, wv = t >> 6;
    for (int p0 = 0; p0 < width; p0 += kQb) {
        // column of the panel and row group, lane indices; the empty asm makes them (and
        // every address derived from them) values of this iteration, so that the compiler
        // does not keep dozens of such addresses live across the whole loop
        int k = t & (kQb - 1), g = t >> 4, lane = t & 63;
        asm volatile("" : "+v"(k), "+v"(g), "+v"(lane));
        const int l16 = lane & 15, l4 = lane >> 4;
        QBuf<S> q;
        if (kind == 0) {
            const int64_t left = m - p0;
            if (left <= 0) break;
            q = qbuf<S>(X + (int64_t)p0 * ld, ld, (int)min(left, (int64_t)(kQGroups * RPT)), nullptr, 0, 0, width);
        } else {
            q = qbuf<S>(X + (int64_t)p0 * ld, ld, min(kQb, width - p0), Y, ldy, min(width, p0 + kQb), width);
        }
        const int na = q.n0 + q.n1;
        const int kb = min(kQb, width - p0);

        // ---- 1. column steps
        // rows past the active ones and columns past the panel (k >= kb) read as 0
        S x[RPT];
        const int kcol = k < kb ? p0 + k : width;
#pragma unroll
        for (int i = 0; i < RPT; i++) x[i] = q.load(g + kQGroups * i, kcol);
        if (t < kQb) L.tau[t] = 0.0;
        int par = 0;
        for (int j = 0; j < kb; j++) {
            if (k == j) {
#pragma unroll
                for (int i = 0; i < RPT; i++) L.f.col[par][g * RPT + i] = x[i];
            }
            if (g == j) L.f.piv[par][k] = (double)x[0];  // the pivot row j is row group j's first row
            __syncthreads();
            S xj[RPT];
#pragma unroll
            for (int i = 0; i < RPT; i++) xj[i] = L.f.col[par][g * RPT + i];
            // rows below the pivot only: row g (i = 0) counts when g > j
            S pp[4] = {S(0), S(0), S(0), S(0)};
            if (g > j) pp[0] = xj[0] * x[0];
#pragma unroll
            for (int i = 1; i < RPT; i++) pp[i & 3] = fma(xj[i], x[i], pp[i & 3]);
            double p = (double)((pp[0] + pp[1]) + (pp[2] + pp[3]));
            p += __shfl_xor(p, 16, 64);
            p += __shfl_xor(p, 32, 64);
            if (l4 == 0) L.f.red[par][wv][k] = p;
            __syncthreads();
            // the wave partials in a fixed order, four at a time
            double sk = 0.0, sj = 0.0;
#pragma unroll
            for (int w = 0; w < kQWaves; w += 4) {
                sk += (L.f.red[par][w][k] + L.f.red[par][w + 1][k]) + (L.f.red[par][w + 2][k] + L.f.red[par][w + 3][k]);
                sj += (L.f.red[par][w][j] + L.f.red[par][w + 1][j]) + (L.f.red[par][w + 2][j] + L.f.red[par][w + 3][j]);
            }
            const double alpha = L.f.piv[par][j], rho = L.f.piv[par][k];
            const double qq = fma(alpha, alpha, sj);
            // a column whose norm below the pivot is not in the normal range is left alone
            const bool ok = sj > 0.0 && qq >= DBL_MIN;
            const double r = q_rsq(ok ? qq : 1.0);
            const double sg = alpha >= 0.0 ? 1.0 : -1.0;
            const double nrm = qq * r;
            const double beta = -sg * nrm;
            const double inv_beta = -sg * r;
            const double scl = q_rcp(ok ? alpha + sg * nrm : 1.0);
            const double tau = 1.0 - alpha * inv_beta;
            if (ok && k > j && k < kb) {
                const double w = rho + scl * sk;
                const S c = (S)(w * inv_beta);
                if (g > j) x[0] = fma(c, xj[0], x[0]);
                else if (g == j) x[0] = (S)(rho - tau * w);
#pragma unroll
                for (int i = 1; i < RPT; i++) x[i] = fma(c, xj[i], x[i]);
            } else if (ok && k == j) {
                if (g > j) x[0] = (S)((double)x[0] * scl);
                else if (g == j) x[0] = (S)beta;
#pragma unroll
                for (int i = 1; i < RPT; i++) x[i] = (S)((double)x[i] * scl);
            }
            if (t == 0) L.tau[j] = ok ? tau : 0.0;
            par ^= 1;
        }

        // ---- 2. R and zeros back into the panel's columns, V to the side buffer
#pragma unroll
        for (int i = 0; i < RPT; i++) {
            const int a = g + kQGroups * i;
            q.store(a, kcol, a <= k ? x[i] : S(0));
            if (a < na) vbuf[(int64_t)a * kQb + k] = k < kb ? (a > k ? x[i] : (a == k ? S(1) : S(0))) : S(0);
        }
        __syncthreads();

        // ---- 3. trailing update
        const int c0 = p0 + kb;
        if (c0 < width) {
            if (width % (16 / (int)sizeof(S)) == 0) q_trail_vec<S>(L, q, vbuf, na, c0, width, wv, lane);
            else q_trail_scalar<S>(L, q, vbuf, na, c0, width, wv, lane);
        }
        __syncthreads();
    }
}

__device__ inline int64_t q_rows_of(const RowSrc &s) { return s.rows_dev ? *s.rows_dev : s.rows_host; }

// dst (width x np FP64) <- the upper triangle of the first min(m, width) rows of src.
template <typename S>
__device__ inline void q_store_tri(double *dst, int np, const S *src, int64_t ld, int64_t m, int width)
{
    for (int e = threadIdx.x; e < width * np; e += kQThreads) {
        const int j = e / np, kk = e - j * np;
        dst[e] = (j < m && kk >= j && kk < width) ? (double)src[(int64_t)j * ld + kk] : 0.0;
    }
}

__device__ inline void q_copy(double *dst, const double *src, int64_t n)
{
    for (int64_t e = threadIdx.x; e < n; e += kQThreads) dst[e] = src[e];
}

// Up to two regions of the same padded width np in one launch, each reduced by a binary
// in-kernel tree: leaf g factorises its rows in place (at most MAXR of them; the number
// of leaves follows the device row count, min(nleaves, ceil(rows / rows_per_leaf)), the
// other workgroups leave at once) and stores its triangle in slot g of level 0; at each
// node the last child to arrive (per-node atomic counter) copies the first child's
// triangle to the parent's slot and merges the second child's triangle into it.  A lone
// child is copied up; the last level's triangle is copied to the root.
// The LDS of a leaf (storage type S) and of the FP64 merges, overlaid.
template <typename S>
union QLdsTree {
    QLds<S> s;
    QLds<double> d;
};

template <typename S>
__global__ __launch_bounds__(kQThreads) void k_wqr_tree(TreeRegion reg0, TreeRegion reg1, int np)
{
    __shared__ QLdsTree<S> U;
    static_assert(sizeof(QLdsTree<S>) <= 160 * 1024, "LDS budget");
    QLds<S> &Ls = U.s;
    QLds<double> &Ld = U.d;
    int g = blockIdx.x;
    const bool second = g >= reg0.nleaves;
    const TreeRegion rg = second ? reg1 : reg0;
    if (second) g -= reg0.nleaves;
    const int width = rg.width;
    const int64_t rows = q_uniform(q_rows_of(rg.src));
    const int64_t want = (rows + rg.rows_per_leaf - 1) / rg.rows_per_leaf;
    const int nleaves = (int)max((int64_t)1, min((int64_t)rg.nleaves, want));
    if (g >= nleaves) return;
    const int64_t tsz = (int64_t)width * np;
    const int64_t chunk = (rows + nleaves - 1) / nleaves;
    const int64_t r_begin = min(rows, (int64_t)g * chunk), r_end = min(rows, r_begin + chunk);
    S *X = (S *)rg.src.p + r_begin * rg.src.ld;
    S *vb = (S *)((char *)rg.vbuf + (int64_t)g * kQVbufBytes);
    q_factor<S, QGeom<S>::RPT>(Ls, 0, X, rg.src.ld, r_end - r_begin, nullptr, 0, width, vb);
    double *R = rg.slots + (int64_t)g * tsz;
    q_store_tri<S>(R, np, X, rg.src.ld, r_end - r_begin, width);

    int node = g, n = nleaves;
    int64_t soff = 0, coff = 0;
    double *vd = (double *)((char *)rg.vbuf + (int64_t)g * kQVbufBytes);
    while (n > 1) {
        const int parent = node >> 1, first = parent << 1;
        const int nchild = min(2, n - first);
        double *P = rg.slots + (soff + n + parent) * tsz;
        __threadfence();  // every thread's stores of its node triangle, before the counter
        __syncthreads();
        if (nchild > 1) {
            if (threadIdx.x == 0) {
                __threadfence();
                Ld.flag = __hip_atomic_fetch_add(&rg.counters[coff + parent], 1, __ATOMIC_ACQ_REL,
                                                 __HIP_MEMORY_SCOPE_AGENT);
                __threadfence();
            }
            __syncthreads();
            if (Ld.flag != 1) return;  // the last child to arrive combines this node
            q_copy(P, rg.slots + (soff + first) * tsz, tsz);
            __syncthreads();
            q_factor<double, kQMergeRpt>(Ld, 1, P, np, width, rg.slots + (soff + first + 1) * tsz, np, width, vd);
        } else {
            q_copy(P, R, tsz);
        }
        R = P;
        node = parent;
        soff += n;
        coff += (n + 1) / 2;
        n = (n + 1) / 2;
    }
    __syncthreads();
    q_copy(rg.root, R, tsz);
}

// top (N x ld1) <- R of [top; bottom], both N-wide upper triangles in FP64; bottom is
// overwritten.  One workgroup.
__global__ __launch_bounds__(kQThreads) void k_wqr_merge(double *top, int64_t ld1, double *bottom, int64_t ld2,
                                                         int width, double *vbuf)
{
    __shared__ QLds<double> Ld;
    q_factor<double, kQMergeRpt>(Ld, 1, top, ld1, width, bottom, ld2, width, vbuf);
}

// dst (n x n, stride ldd) <- the triangle src (w x w, stride lds) placed at rows [0, w)
// and columns [off, off + w), zeros elsewhere.
__global__ void k_wqr_pad(const double *src, int64_t lds, int w, int off, double *dst, int64_t ldd, int n)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * n) return;
    const int i = (int)(e / n), c = (int)(e - (int64_t)i * n);
    const int kk = c - off;
    dst[(int64_t)i * ldd + c] = (i < w && kk >= i && kk < w) ? src[(int64_t)i * lds + kk] : 0.0;
}

}  // namespace

int64_t wqr_leaf_rows(int in_f64) { return in_f64 ? QGeom<double>::MAXR : QGeom<float>::MAXR; }
int64_t wqr_vbuf_bytes() { return kQVbufBytes; }

hipError_t launch_wqr_tree(int np, int in_f64, const TreeRegion *regs, int nreg, hipStream_t s)
{
    if (nreg < 1 || nreg > 2 || (np != 128 && np != 256 && np != 512)) return hipErrorInvalidValue;
    const TreeRegion r0 = regs[0];
    const TreeRegion r1 = nreg > 1 ? regs[1] : TreeRegion{};
    const unsigned grid = (unsigned)(r0.nleaves + r1.nleaves);
    if (in_f64) k_wqr_tree<double><<<grid, kQThreads, 0, s>>>(r0, r1, np);
    else k_wqr_tree<float><<<grid, kQThreads, 0, s>>>(r0, r1, np);
    return hipGetLastError();
}

hipError_t launch_wqr_merge(double *top, int64_t ld1, double *bottom, int64_t ld2, int width, double *vbuf,
                            hipStream_t s)
{
    if (width < 1 || width > 512) return hipErrorInvalidValue;
    k_wqr_merge<<<1, kQThreads, 0, s>>>(top, ld1, bottom, ld2, width, vbuf);
    return hipGetLastError();
}

hipError_t launch_wqr_pad(const double *src, int64_t lds, int w, int off, double *dst, int64_t ldd, int n,
                          hipStream_t s)
{
    const int64_t nn = (int64_t)n * n;
    k_wqr_pad<<<(unsigned)((nn + 255) / 256), 256, 0, s>>>(src, lds, w, off, dst, ldd, n);
    return hipGetLastError();
}

}  // namespace figaro
