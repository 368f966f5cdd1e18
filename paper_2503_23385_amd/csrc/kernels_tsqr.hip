// Householder TSQR of the compact matrix (the QR step of the paper's
// pipeline, Experiments section: dense Householder QR of the concatenated
// heads and tails; here done as a tall-skinny reduction instead of a
// library geqrf).
//
// Each workgroup owns one N x N upper triangle R (packed in LDS) and streams
// its share of rows through it in blocks X of BR rows:
//     R <- triu(QR([R; X])).
// Reflector j of a step involves only row j of R and column j of X
// (structured TSQR): with alpha = R_jj and s = |X_:j|^2,
//     beta = -sign(alpha) sqrt(alpha^2 + s),  tau = (beta - alpha) / beta,
//     v = X_:j / (alpha - beta),  w_k = R_jk + v . X_:k,
//     R_jk -= tau w_k,  X_:k -= tau w_k v          (k > j),  R_jj = beta.
// Q is never formed: only R is wanted.  Thread layout: wave w owns columns
// [w*CW, (w+1)*CW); lane (k, q) keeps RPT rows of column k of X in registers,
// so every reduction over rows is a shuffle inside one wave and the only
// cross-wave exchange per column is the reflector v (one LDS broadcast and
// one barrier per column, double-buffered).
//
// The same kernel reduces stacked triangles (tree levels) and the final
// [R_1 ; 0 | R_2] merge of the two compact-matrix regions; sign
// normalisation of the root is a separate tiny kernel.
#include "common.h"

namespace figaro {
namespace {

constexpr int kTsqrThreads = 256;

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

template <int NP, typename Tin, typename Tacc>
__global__ __launch_bounds__(kTsqrThreads) void k_tsqr_stream(RowSrc s0, RowSrc s1, int nsrc,
                                                              int width, int tri_rows,
                                                              double *tri_out, int64_t tri_stride)
{
    constexpr int CW = NP / 4 > 0 ? NP / 4 : 1;  // columns per wave
    constexpr int Q = 64 / CW;                   // row groups per column
    constexpr int RPT = 16;                      // rows per thread per block
    constexpr int BR = Q * RPT;                  // rows per block
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int k = wave * CW + (lane % CW);
    const int q = lane / CW;

    __shared__ Tacc Rp[packed_size(NP)];
    __shared__ Tacc vbuf[2][BR];
    __shared__ double sc[2][2];

    for (int i = tid; i < packed_size(NP); i += kTsqrThreads) Rp[i] = Tacc(0);

    const int64_t rows0 = src_rows(s0);
    const int64_t total = rows0 + (nsrc > 1 ? src_rows(s1) : 0);
    int64_t chunk = (total + gridDim.x - 1) / gridDim.x;
    chunk = ((chunk + BR - 1) / BR) * BR;
    const int64_t r_begin = (int64_t)blockIdx.x * chunk;
    const int64_t r_end = min(total, r_begin + chunk);
    __syncthreads();

    int it = 0;  // global column-step counter: parity of the LDS buffers
    for (int64_t rb = r_begin; rb < r_end; rb += BR) {
        Tacc x[RPT];
#pragma unroll
        for (int i = 0; i < RPT; i++) {
            const int64_t r = rb + q * RPT + i;
            Tacc v = Tacc(0);
            if (r < r_end && k < width) {
                if (r < rows0) v = load_src<Tin, Tacc>(s0, r, k);
                else v = load_src<Tin, Tacc>(s1, r - rows0, k);
            }
            x[i] = v;
        }
        // Rows of a stacked triangle are zero left of their index within it.
        int jstart = 0;
        if (tri_rows > 0) {
            const int64_t off = rb % tri_rows;
            if (off + BR <= tri_rows) jstart = (int)off;
        }
        for (int j = jstart; j < width; j++, it++) {
            const int buf = it & 1;
            if (wave == j / CW) {
                double pn = 0.0;
#pragma unroll
                for (int i = 0; i < RPT; i++) pn += (double)x[i] * (double)x[i];
#pragma unroll
                for (int off = CW; off < 64; off <<= 1) pn += shfl_xor_t(pn, off);
                const double s = __shfl(pn, j % CW, 64);
                const double alpha = (double)Rp[pidx(NP, j, j)];
                double tau = 0.0, beta = alpha, scl = 0.0;
                if (s > 0.0) {
                    const double nrm = sqrt(alpha * alpha + s);
                    beta = alpha >= 0.0 ? -nrm : nrm;
                    tau = (beta - alpha) / beta;
                    scl = 1.0 / (alpha - beta);
                }
                if (k == j) {
#pragma unroll
                    for (int i = 0; i < RPT; i++) vbuf[buf][q * RPT + i] = (Tacc)((double)x[i] * scl);
                }
                if (lane == 0) {
                    sc[buf][0] = tau;
                    sc[buf][1] = beta;
                }
            }
            __syncthreads();
            const double tau = sc[buf][0];
            if (tau != 0.0) {
                const Tacc rjk = (k > j && k < width) ? Rp[pidx(NP, j, k)] : Tacc(0);
                Tacc dot = Tacc(0);
#pragma unroll
                for (int i = 0; i < RPT; i++) dot += vbuf[buf][q * RPT + i] * x[i];
#pragma unroll
                for (int off = CW; off < 64; off <<= 1) dot += shfl_xor_t(dot, off);
                if (k > j && k < width) {
                    const Tacc w = rjk + dot;
                    const Tacc tw = (Tacc)tau * w;
#pragma unroll
                    for (int i = 0; i < RPT; i++) x[i] -= vbuf[buf][q * RPT + i] * tw;
                    if (q == 0) Rp[pidx(NP, j, k)] = rjk - tw;
                }
                if (k == j && q == 0) Rp[pidx(NP, j, j)] = (Tacc)sc[buf][1];
            }
        }
    }
    __syncthreads();
    // Triangle out: `width` rows of NP columns (zeros left of the diagonal).
    double *out = tri_out + (int64_t)blockIdx.x * tri_stride;
    for (int e = tid; e < width * NP; e += kTsqrThreads) {
        const int j = e / NP, kk = e - j * NP;
        out[e] = (kk >= j && kk < width) ? (double)Rp[pidx(NP, j, kk)] : 0.0;
    }
}

__device__ inline double readlane_f64(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}
__device__ inline float readlane_f32(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ inline double readlane_t(double v, int l) { return readlane_f64(v, l); }
__device__ inline float readlane_t(float v, int l) { return readlane_f32(v, l); }

// One wave per triangle (widths up to 64): lane (k, h) holds RPT rows of column k of the
// block for row set h (H = 64 / NP row sets).  Column j of the block is broadcast through a
// per-wave LDS slot; all reductions stay inside the wave, so there is no workgroup barrier.
// With d_k = x_j . x_k (d_j = |x_j|^2) and p = beta (alpha - beta):
//     w_k = R_jk + d_k / (alpha - beta),  R_jk -= tau w_k,  x_k += (w_k / beta) x_j,
// which is the reflector update above with tau * scale = -1 / beta folded in.
constexpr int kWavesPerBlock = 4;

template <int NP, typename Tin, typename Tacc, int RPT>
__global__ __launch_bounds__(64 * kWavesPerBlock) void k_tsqr_wave(RowSrc s0, RowSrc s1, int nsrc,
                                                                  int width, int tri_rows, int ntri,
                                                                  double *tri_out, int64_t tri_stride)
{
    constexpr int H = NP >= 64 ? 1 : 64 / NP;
    constexpr int BR = H * RPT;
    constexpr int PS = packed_size(NP);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int gw = blockIdx.x * kWavesPerBlock + wv;
    const int k = lane % NP;
    const int h = lane / NP;
    __shared__ Tacc Rs[kWavesPerBlock][PS];
    __shared__ __align__(16) Tacc Xs[kWavesPerBlock][BR];
    if (gw >= ntri) return;  // waves are independent: no block-level barrier follows
    Tacc *Rp = Rs[wv];
    Tacc *xb = Xs[wv] + h * RPT;
    for (int i = lane; i < PS; i += 64) Rp[i] = Tacc(0);

    const int64_t rows0 = src_rows(s0);
    const int64_t total = rows0 + (nsrc > 1 ? src_rows(s1) : 0);
    int64_t chunk = (total + ntri - 1) / ntri;
    chunk = ((chunk + BR - 1) / BR) * BR;
    const int64_t r_begin = (int64_t)gw * chunk;
    const int64_t r_end = min(total, r_begin + chunk);
    const bool col_ok = k < width;

    for (int64_t rb = r_begin; rb < r_end; rb += BR) {
        Tacc x[RPT];
#pragma unroll
        for (int i = 0; i < RPT; i++) {
            const int64_t r = rb + h * RPT + i;
            Tacc v = Tacc(0);
            if (r < r_end && col_ok) {
                if (r < rows0) v = load_src<Tin, Tacc>(s0, r, k);
                else v = load_src<Tin, Tacc>(s1, r - rows0, k);
            }
            x[i] = v;
        }
        int jstart = 0;
        if (tri_rows > 0) {
            const int64_t off = rb % tri_rows;
            if (off + BR <= tri_rows) jstart = (int)off;
        }
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
            Tacc d0 = Tacc(0), d1 = Tacc(0);
#pragma unroll
            for (int i = 0; i < RPT; i += 2) {
                d0 += xj[i] * x[i];
                if (i + 1 < RPT) d1 += xj[i + 1] * x[i + 1];
            }
            Tacc d = d0 + d1;
#pragma unroll
            for (int off = NP; off < 64; off <<= 1) d += shfl_xor_t(d, off);
            double s;
            if constexpr (sizeof(Tacc) == 8) {
                s = readlane_t(d, j);
            } else {
                // reflector scalars in FP64 for the FP32 form
                double sd = 0.0;
#pragma unroll
                for (int i = 0; i < RPT; i++) sd += (double)xj[i] * (double)xj[i];
#pragma unroll
                for (int off = NP; off < 64; off <<= 1) sd += shfl_xor_t(sd, off);
                s = readlane_f64(sd, j);
            }
            if (s > 0.0) {
                const double nrm = sqrt(alpha * alpha + s);
                const double beta = alpha >= 0.0 ? -nrm : nrm;
                const double amb = alpha - beta;
                const double rp = 1.0 / (beta * amb);
                const double inv_beta = amb * rp;
                const double scl = beta * rp;
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
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    double *out = tri_out + (int64_t)gw * tri_stride;
    for (int e = lane; e < width * NP; e += 64) {
        const int j = e / NP, kk = e - j * NP;
        out[e] = (kk >= j && kk < width) ? (double)Rp[pidx(NP, j, kk)] : 0.0;
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
hipError_t launch_np(int acc_f64, int in_f64, RowSrc s0, RowSrc s1, int nsrc, int width, int tri_rows,
                     int nwg, double *tri, int64_t stride, hipStream_t s)
{
    if constexpr (NP <= 64) {
        const unsigned grid = (unsigned)((nwg + kWavesPerBlock - 1) / kWavesPerBlock);
#define FIGARO_WAVE(TI, TA) \
    k_tsqr_wave<NP, TI, TA, 16><<<grid, 64 * kWavesPerBlock, 0, s>>>(s0, s1, nsrc, width, tri_rows, nwg, tri, stride)
        if (acc_f64) {
            if (in_f64) FIGARO_WAVE(double, double);
            else FIGARO_WAVE(float, double);
        } else {
            if (in_f64) FIGARO_WAVE(double, float);
            else FIGARO_WAVE(float, float);
        }
#undef FIGARO_WAVE
        return hipGetLastError();
    }
    if (acc_f64) {
        if constexpr (packed_size(NP) * 8 + 2 * 16 * (256 / NP) * 8 <= 160 * 1024) {
            if (in_f64)
                k_tsqr_stream<NP, double, double><<<nwg, kTsqrThreads, 0, s>>>(s0, s1, nsrc, width, tri_rows, tri, stride);
            else
                k_tsqr_stream<NP, float, double><<<nwg, kTsqrThreads, 0, s>>>(s0, s1, nsrc, width, tri_rows, tri, stride);
        } else {
            return hipErrorInvalidValue;
        }
    } else {
        if (in_f64)
            k_tsqr_stream<NP, double, float><<<nwg, kTsqrThreads, 0, s>>>(s0, s1, nsrc, width, tri_rows, tri, stride);
        else
            k_tsqr_stream<NP, float, float><<<nwg, kTsqrThreads, 0, s>>>(s0, s1, nsrc, width, tri_rows, tri, stride);
    }
    return hipGetLastError();
}

}  // namespace

int tsqr_padded_width(int n)
{
    if (n <= 0) return 0;
    int np = 4;
    while (np < n) np <<= 1;
    return np <= 256 ? np : 0;
}

int tsqr_block_rows(int np)
{
    if (np <= 64) return (64 / np) * 16;  // wave kernel: row sets x rows per thread
    return (256 / np) * 16;               // workgroup kernel
}

hipError_t launch_tsqr_stream(int np, int acc_f64, int in_f64, RowSrc s0, RowSrc s1, int nsrc,
                              int width, int tri_rows, int nwg, double *tri,
                              int64_t tri_stride, hipStream_t s)
{
    switch (np) {
    case 4: return launch_np<4>(acc_f64, in_f64, s0, s1, nsrc, width, tri_rows, nwg, tri, tri_stride, s);
    case 8: return launch_np<8>(acc_f64, in_f64, s0, s1, nsrc, width, tri_rows, nwg, tri, tri_stride, s);
    case 16: return launch_np<16>(acc_f64, in_f64, s0, s1, nsrc, width, tri_rows, nwg, tri, tri_stride, s);
    case 32: return launch_np<32>(acc_f64, in_f64, s0, s1, nsrc, width, tri_rows, nwg, tri, tri_stride, s);
    case 64: return launch_np<64>(acc_f64, in_f64, s0, s1, nsrc, width, tri_rows, nwg, tri, tri_stride, s);
    case 128: return launch_np<128>(acc_f64, in_f64, s0, s1, nsrc, width, tri_rows, nwg, tri, tri_stride, s);
    case 256: return launch_np<256>(acc_f64, in_f64, s0, s1, nsrc, width, tri_rows, nwg, tri, tri_stride, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sign_normalise(const void *Rin, int in_f64, int64_t ldin, int n, double *R,
                                 int64_t ldr, hipStream_t s)
{
    (void)in_f64;
    k_sign_normalise<<<n, 64, 0, s>>>((const double *)Rin, ldin, n, R, ldr);
    return hipGetLastError();
}

}  // namespace figaro
