// Singular values of R by one-sided (Hestenes) Jacobi in FP64.
//
// The singular values of the join matrix equal those of R (Related Works:
// SVD through QR); the paper obtains them with a dense SVD of R.  Here one
// workgroup keeps R's columns in LDS and orthogonalises column pairs with
// plane rotations until every pair satisfies |c_p . c_q| <= n 2^-53 |c_p||c_q|.
// Pairs are visited in a round-robin (circle) order: each of the n-1 steps of
// a sweep rotates n/2 disjoint pairs in parallel, so a sweep still meets
// every pair once.  For a pair with alpha = |c_p|^2, beta = |c_q|^2,
// gamma = c_p . c_q, the rotation that zeroes gamma with |angle| <= pi/4 is
//     u = beta - alpha, v = 2 gamma, h = sqrt(u^2 + v^2),
//     c = sqrt((1 + |u|/h) / 2),  s = sign(u) v / (2 h c),
//     (c_p, c_q) <- (c c_p - s c_q, s c_p + c c_q)
// (the same rotation as t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)) with
// zeta = u / v, written with two reciprocal square roots and no division).
// sigma_k = |c_k| after convergence, sorted descending.
//
// A lane group (4 to 16 lanes, so that a step fits four waves) shares a pair and keeps
// its two columns in registers for the whole step; the three dot products are
// reduced with DPP moves inside the group; one workgroup barrier separates the
// steps.  The width is a template parameter so every loop over rows is unrolled.
#include <float.h>
#include <limits.h>

#include <cstdlib>

#include "common.h"

namespace figaro {
namespace {

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

// DPP move of a double (every lane reads an in-range source for the patterns used here).
template <int CTRL>
__device__ inline double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
// Sum over an aligned group of LP (4, 8 or 16) lanes with DPP: xor 1, xor 2,
// then for 8 and 16 the half-row mirror (lane i <-> 7 - i, swapping the quads of
// 8 lanes) and for 16 the row mirror (lane i <-> 15 - i, swapping the halves).
template <int LP>
__device__ inline double group_sum(double v)
{
    static_assert(LP == 4 || LP == 8 || LP == 16, "group of 4, 8 or 16 lanes");
    v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    if constexpr (LP >= 8) v += dpp_f64<0x141>(v);  // row_half_mirror
    if constexpr (LP == 16) v += dpp_f64<0x140>(v);  // row_mirror
    return v;
}

// Sum over the 64 lanes of a wave, the same value in every lane (defined below).
__device__ inline double wave_sum(double v);

// Rotation (c, s) that zeroes gamma for the pair (alpha, beta, gamma), gamma != 0.
// u and v are scaled by a power of two first so that u^2 + v^2 neither overflows
// nor underflows (c and s depend only on their ratio).
__device__ inline void jacobi_rotation(double alpha, double beta, double gamma, double &c, double &s)
{
    double u = beta - alpha, v = 2.0 * gamma;
    const int e = ilogb(fmax(fabs(u), fabs(v)));
    u = ldexp(u, -e);
    v = ldexp(v, -e);
    const double rh = rsq_refined(fma(u, u, v * v));  // 1 / h
    const double x = fma(0.5 * fabs(u), rh, 0.5);      // (1 + cos 2 theta) / 2, in [1/2, 1]
    const double rc = rsq_refined(x);                   // 1 / c
    c = x * rc;
    s = (u >= 0.0 ? 0.5 : -0.5) * v * rh * rc;
}

// NPC: padded (even, power of two) column count; columns n..NPC-1 are zero.
// LP: lanes per pair (4, 8 or 16, at most NPC).  Fewer lanes per pair issue the
// per-pair reductions and the rotation, which every lane of a group repeats, on
// fewer waves; more lanes give more waves to hide latency with.
template <int NPC, int LP>
struct JacobiGeom {
    static_assert(LP == 4 || LP == 8 || LP == 16, "lanes per pair");
    static_assert(LP <= NPC, "at least one row per lane");
    static constexpr int RPL = NPC / LP;           // rows per lane
    static constexpr int PAIRS = NPC / 2;
    static constexpr int THREADS = PAIRS * LP < 64 ? 64 : PAIRS * LP;
    // Column stride: column k starts LP doubles further along the 32-double bank
    // window than column k - 1, so the pairs of one wave, whose columns are
    // consecutive in the circle order, read disjoint banks.
    static constexpr int LDC = NPC + LP;
};

// With Vc (global, NPC columns of NPC doubles, column-major) the rotations are also
// applied to the columns of V, which starts as the identity: R V = U Sigma, and V (n x n,
// ld ldv) receives the right singular vectors in the order of sigma.
template <int NPC, int LP>
__device__ __forceinline__ void jacobi_lds_body(const double *R, int n, int64_t ldr, double *sigma, int max_sweeps,
                                int32_t *sweeps_out, double *Vc = nullptr, double *V = nullptr, int64_t ldv = 0)
{
    using Gm = JacobiGeom<NPC, LP>;
    constexpr int RPL = Gm::RPL, PAIRS = Gm::PAIRS, LDC = Gm::LDC;
    __shared__ double C[NPC * LDC];  // column k at C[k * LDC]
    __shared__ double sv[NPC];
    __shared__ int s_rot;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    staged_copy<8, double>(
        NPC * NPC, tid, nthr,
        [&](int e) {
            const int k = e / NPC, i = e - k * NPC;
            return R[(int64_t)(i < n ? i : n - 1) * ldr + (k < n ? k : n - 1)];
        },
        [&](int e, double v) {
            const int k = e / NPC, i = e - k * NPC;
            C[k * LDC + i] = (k < n && i < n) ? v : 0.0;
        });
    const int pair = tid / LP, sub = tid % LP;
    // every lane has a pair unless the pairs fill less than one wave
    const bool active = PAIRS * LP >= Gm::THREADS || pair < PAIRS;
    const double tol2 = ((double)n * 0x1p-53) * ((double)n * 0x1p-53);
    constexpr int M = NPC - 1;
    int sweeps = 0;
    // Scale by a power of two so that the largest |entry| lies in [1, 2): squared norms stay in range.
    __shared__ int s_exp;
    if (tid == 0) s_exp = INT_MIN;
    __syncthreads();
    {
        double m = 0.0;
        for (int e = tid; e < NPC * NPC; e += nthr) m = fmax(m, fabs(C[(e / NPC) * LDC + e % NPC]));
        if (m > 0.0) atomicMax(&s_exp, ilogb(m));
    }
    __syncthreads();
    const int ex = s_exp == INT_MIN ? 0 : s_exp;
    for (int e = tid; e < NPC * NPC; e += nthr) {
        double &x = C[(e / NPC) * LDC + e % NPC];
        x = ldexp(x, -ex);
        if (Vc) Vc[e] = (e / NPC == e % NPC) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int sweep = 0; sweep < max_sweeps; sweep++) {
        if (tid == 0) s_rot = 0;
        __syncthreads();
        // pair slots of the circle order: (step, NPC-1) for pair 0, else
        // ((step + pair) mod M, (step - pair) mod M), advanced by one step at a time
        int pa = pair == 0 ? 0 : pair % M, qa = pair == 0 ? NPC - 1 : (M - pair % M) % M;
        for (int step = 0; step < M; step++) {
            // (p, q) and (q, p) give the same rotated pair, so slots are not reordered
            const int p = active ? pa : 0, q = active ? qa : 0;
            pa = pa + 1 == M ? 0 : pa + 1;
            if (pair != 0) qa = qa + 1 == M ? 0 : qa + 1;
            double *cp = C + p * LDC + sub, *cq = C + q * LDC + sub;
            double xp[RPL], xq[RPL];
#pragma unroll
            for (int r = 0; r < RPL; r++) {
                xp[r] = active ? cp[r * LP] : 0.0;
                xq[r] = active ? cq[r * LP] : 0.0;
            }
            // up to four independent partial sums per dot product (short FMA chains)
            constexpr int NA = RPL >= 4 ? 4 : RPL;
            double pa_[NA], pb_[NA], pg_[NA];
#pragma unroll
            for (int t = 0; t < NA; t++) pa_[t] = pb_[t] = pg_[t] = 0.0;
#pragma unroll
            for (int r = 0; r < RPL; r++) {
                pa_[r % NA] = fma(xp[r], xp[r], pa_[r % NA]);
                pb_[r % NA] = fma(xq[r], xq[r], pb_[r % NA]);
                pg_[r % NA] = fma(xp[r], xq[r], pg_[r % NA]);
            }
#pragma unroll
            for (int t = NA / 2; t >= 1; t /= 2) {
#pragma unroll
                for (int u = 0; u < t; u++) {
                    pa_[u] += pa_[u + t];
                    pb_[u] += pb_[u + t];
                    pg_[u] += pg_[u + t];
                }
            }
            double a = group_sum<LP>(pa_[0]);
            double b = group_sum<LP>(pb_[0]);
            double g = group_sum<LP>(pg_[0]);
            if (active && g * g > tol2 * a * b) {
                double c, s;
                jacobi_rotation(a, b, g, c, s);
#pragma unroll
                for (int r = 0; r < RPL; r++) {
                    cp[r * LP] = c * xp[r] - s * xq[r];
                    cq[r * LP] = s * xp[r] + c * xq[r];
                }
                if (Vc) {
                    double *vp = Vc + p * NPC + sub, *vq = Vc + q * NPC + sub;
                    double yp[RPL], yq[RPL];
#pragma unroll
                    for (int r = 0; r < RPL; r++) {
                        yp[r] = vp[r * LP];
                        yq[r] = vq[r * LP];
                    }
#pragma unroll
                    for (int r = 0; r < RPL; r++) {
                        vp[r * LP] = c * yp[r] - s * yq[r];
                        vq[r * LP] = s * yp[r] + c * yq[r];
                    }
                }
                if (sub == 0) s_rot = 1;
            }
            __syncthreads();
        }
        sweeps++;
        const int any = s_rot;
        __syncthreads();
        if (!any) break;
    }
    for (int k = tid; k < n; k += nthr) {
        double acc = 0.0;
        for (int i = 0; i < NPC; i++) acc += C[k * LDC + i] * C[k * LDC + i];
        sv[k] = ldexp(sqrt(acc), ex);
    }
    __syncthreads();
    for (int k = tid; k < n; k += nthr) {
        const double v = sv[k];
        int rank = 0;
        for (int j = 0; j < n; j++) {
            const double u = sv[j];
            rank += (u > v) || (u == v && j < k);
        }
        sigma[rank] = v;
        if (V)
            for (int i = 0; i < n; i++) V[(int64_t)i * ldv + rank] = Vc[k * NPC + i];
    }
    if (tid == 0 && sweeps_out) *sweeps_out = sweeps;
}

template <int NPC, int LP>
__global__ __launch_bounds__((JacobiGeom<NPC, LP>::THREADS))
void k_jacobi_lds(const double *R, int n, int64_t ldr, double *sigma, int max_sweeps, int32_t *sweeps_out)
{
    jacobi_lds_body<NPC, LP>(R, n, ldr, sigma, max_sweeps, sweeps_out);
}

template <int NPC, int LP>
__global__ __launch_bounds__((JacobiGeom<NPC, LP>::THREADS))
void k_jacobi_v(const double *R, int n, int64_t ldr, double *sigma, int max_sweeps, int32_t *sweeps_out, double *Vc,
                double *V, int64_t ldv)
{
    jacobi_lds_body<NPC, LP>(R, n, ldr, sigma, max_sweeps, sweeps_out, Vc, V, ldv);
}

// Lanes per pair for a width class: FIGARO_JACOBI_LP (4, 8 or 16) when it is set and
// valid for the class, else the measured default.
int jacobi_lanes(int npc)
{
    static const int forced = [] {
        const char *v = std::getenv("FIGARO_JACOBI_LP");
        return v ? std::atoi(v) : 0;
    }();
    if ((forced == 4 || forced == 8 || forced == 16) && forced <= npc) return forced;
    return npc <= 8 ? npc : 16;
}

template <int NPC>
hipError_t launch_npc(const double *R, int n, int64_t ldr, double *sigma, int max_sweeps,
                      int32_t *sweeps_out, hipStream_t s)
{
    const int lp = jacobi_lanes(NPC);
    if constexpr (NPC >= 16) {
        if (lp == 16) {
            k_jacobi_lds<NPC, 16><<<1, JacobiGeom<NPC, 16>::THREADS, 0, s>>>(R, n, ldr, sigma, max_sweeps, sweeps_out);
            return hipGetLastError();
        }
    }
    if (lp == 8) {
        k_jacobi_lds<NPC, 8><<<1, JacobiGeom<NPC, 8>::THREADS, 0, s>>>(R, n, ldr, sigma, max_sweeps, sweeps_out);
        return hipGetLastError();
    }
    k_jacobi_lds<NPC, 4><<<1, JacobiGeom<NPC, 4>::THREADS, 0, s>>>(R, n, ldr, sigma, max_sweeps, sweeps_out);
    return hipGetLastError();
}

template <int NPC>
hipError_t launch_v_npc(const double *R, int n, int64_t ldr, double *sigma, int max_sweeps, int32_t *sweeps_out,
                        double *Vc, double *V, int64_t ldv, hipStream_t s)
{
    constexpr int LP = NPC <= 8 ? NPC : 16;
    k_jacobi_v<NPC, LP><<<1, JacobiGeom<NPC, LP>::THREADS, 0, s>>>(R, n, ldr, sigma, max_sweeps, sweeps_out, Vc, V,
                                                                    ldv);
    return hipGetLastError();
}

// ------------------------------------------------------------------ block Jacobi (n up to 512)
//
// For wider R the columns live in global memory (column-major, NPC x NPC) and
// are split into blocks of 16.  A persistent grid of NPC / 32 workgroups runs
// a round-robin over block pairs: in each round every workgroup loads one pair
// of blocks (32 columns C) into LDS, forms G = C^T C on the matrix cores, applies
// one cyclic sweep of the pair rotations to G (each rotation computed from
// G_pp, G_qq, G_pq, exactly as from the columns, with G <- J^T G J) while
// accumulating them in V, then C <- C V on the matrix cores, writes the columns
// back, and meets the others at a grid barrier.  Each round starts from a G formed
// afresh from the columns, so the rotations' rounding does not accumulate there.  nb - 1 rounds make an outer sweep in which every column pair meets
// at least once; the iteration stops after an outer sweep without rotations.
// Every wait is bounded: a barrier that does not complete within the spin limit
// marks the run as timed out and every workgroup leaves.

constexpr int kBlk = 16;            // columns per block
constexpr int kBlkThreads = 1024;
constexpr int kBlkWaves = kBlkThreads / 64;
enum : int { CTRL_SWEEPS = 0, CTRL_BAR = 1, CTRL_FLAG = 2, CTRL_TIMEOUT = 5, CTRL_EXP = 6, CTRL_WORDS = 8 };
constexpr int kSpinLimit = 1 << 22;

__global__ void k_jacobi_blk_init(const double *R, int n, int64_t ldr, double *C, int npc, int32_t *ctrl)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < CTRL_WORDS) ctrl[e] = 0;
    if (e >= (int64_t)npc * npc) return;
    const int k = (int)(e / npc), i = (int)(e - (int64_t)k * npc);
    C[e] = (k < n && i < n) ? R[(int64_t)i * ldr + k] : 0.0;
}

// All workgroups of the grid meet; false if the wait timed out (then every caller leaves).
__device__ inline bool grid_barrier(int32_t *ctrl, int target)
{
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicAdd(&ctrl[CTRL_BAR], 1);
        int ok = 1, spins = 0;
        while (atomicAdd(&ctrl[CTRL_BAR], 0) < target) {
            if (atomicAdd(&ctrl[CTRL_TIMEOUT], 0) != 0 || ++spins > kSpinLimit) {
                atomicExch(&ctrl[CTRL_TIMEOUT], 1);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

template <int NPC>
__global__ __launch_bounds__(kBlkThreads) void k_jacobi_blk(double *C, int n, int max_sweeps, int32_t *ctrl)
{
    constexpr int LOC = 2 * kBlk, LDC = NPC + 1;  // odd stride: a column-strided access is conflict free
    typedef double d4 __attribute__((ext_vector_type(4)));
    __shared__ double Cs[LOC * LDC];
    __shared__ double Gs[LOC][LOC + 1], Vs[LOC][LOC + 1];
    __shared__ double rc_[LOC / 2], rs_[LOC / 2];
    __shared__ int rp_[LOC / 2], rq_[LOC / 2];
    __shared__ int s_rot;
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, l16 = lane & 15, l4 = lane >> 4;
    const int P = gridDim.x, w = blockIdx.x;
    const int nb = 2 * P, M = nb - 1;
    const double tol2 = ((double)n * 0x1p-53) * ((double)n * 0x1p-53);
    int epoch = 0, sweeps = 0;
    bool alive = true;
    // Power-of-two scale (largest |entry| into [1, 2)), the same in every workgroup; each
    // block is scaled by the workgroup that loads it in the first round.
    __shared__ int s_exp;
    if (tid == 0) s_exp = INT_MIN;
    __syncthreads();
    {
        double m = 0.0;
        for (int64_t e = tid; e < (int64_t)NPC * NPC; e += kBlkThreads) m = fmax(m, fabs(C[e]));
        if (m > 0.0) atomicMax(&s_exp, ilogb(m));
    }
    __syncthreads();
    const int ex = s_exp == INT_MIN ? 0 : s_exp;
    if (w == 0 && tid == 0) ctrl[CTRL_EXP] = ex;
    // every workgroup has read the unscaled columns before any is written back
    epoch++;
    alive = grid_barrier(ctrl, epoch * P);
    for (int sweep = 0; sweep < max_sweeps && alive; sweep++) {
        if (w == 0 && tid == 0) ctrl[CTRL_FLAG + (sweep + 1) % 3] = 0;
        for (int round = 0; round < M; round++) {
            const int bp = w == 0 ? round : (round + w) % M;
            const int bq = w == 0 ? nb - 1 : (round - w + M) % M;
            for (int e = tid; e < LOC * NPC; e += kBlkThreads) {
                const int l = e / NPC, i = e - l * NPC;
                const int col = (l < kBlk ? bp * kBlk + l : bq * kBlk + (l - kBlk));
                const double x = C[(int64_t)col * NPC + i];
                Cs[l * LDC + i] = (sweep == 0 && round == 0) ? ldexp(x, -ex) : x;
            }
            if (tid == 0) s_rot = 0;
            __syncthreads();
            // 1. G = C^T C of the 32 local columns on the FP64 matrix cores (waves 0..2 form
            //    the tiles (0,0), (0,1), (1,1) over all rows); V = I
            if (wv < 3) {
                const int ti = wv == 2 ? 1 : 0, tj = wv == 0 ? 0 : 1;
                const double *ca = Cs + (ti * 16 + l16) * LDC, *cb = Cs + (tj * 16 + l16) * LDC;
                d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
                for (int k0 = 0; k0 < NPC; k0 += 4)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[k0 + l4], cb[k0 + l4], acc, 0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int i = ti * 16 + l4 + 4 * r, j = tj * 16 + l16;
                    Gs[i][j] = acc[r];
                    if (ti != tj) Gs[j][i] = acc[r];
                }
            }
            for (int e = tid; e < LOC * LOC; e += kBlkThreads) Vs[e / LOC][e % LOC] = (e / LOC == e % LOC) ? 1.0 : 0.0;
            __syncthreads();
            // 2. one cyclic sweep of the same pair rotations on G = C^T C (the rotation of a
            //    pair from (G_pp, G_qq, G_pq), as from the columns themselves), G <- J^T G J,
            //    V <- V J; 16 disjoint pairs per step
            constexpr int ML = LOC - 1;
            for (int step = 0; step < ML; step++) {
                if (tid < LOC / 2) {
                    const int pr = tid;
                    int p = pr == 0 ? step % ML : (pr + step) % ML;
                    int q = pr == 0 ? LOC - 1 : (ML - pr + step) % ML;
                    if (p > q) { const int t = p; p = q; q = t; }
                    const double a = Gs[p][p], b = Gs[q][q], g = Gs[p][q];
                    double c = 1.0, sn = 0.0;
                    if (g * g > tol2 * a * b) {
                        jacobi_rotation(a, b, g, c, sn);
                        s_rot = 1;
                    }
                    rp_[pr] = p;
                    rq_[pr] = q;
                    rc_[pr] = c;
                    rs_[pr] = sn;
                }
                __syncthreads();
                {
                    const int u = tid & 511, pr = u >> 5, x = u & 31;
                    const int p = rp_[pr], q = rq_[pr];
                    const double c = rc_[pr], sn = rs_[pr];
                    if (tid < 512) {  // rows p, q of G
                        const double gp = Gs[p][x], gq = Gs[q][x];
                        Gs[p][x] = c * gp - sn * gq;
                        Gs[q][x] = sn * gp + c * gq;
                    } else {          // columns p, q of V
                        const double vp = Vs[x][p], vq = Vs[x][q];
                        Vs[x][p] = c * vp - sn * vq;
                        Vs[x][q] = sn * vp + c * vq;
                    }
                }
                __syncthreads();
                if (tid < 512) {      // columns p, q of G
                    const int pr = tid >> 5, x = tid & 31;
                    const int p = rp_[pr], q = rq_[pr];
                    const double c = rc_[pr], sn = rs_[pr];
                    const double gp = Gs[x][p], gq = Gs[x][q];
                    Gs[x][p] = c * gp - sn * gq;
                    Gs[x][q] = sn * gp + c * gq;
                }
                __syncthreads();
            }
            // 3. C <- C V on the matrix cores, in place: wave wv owns rows [32 wv, 32 wv + 32)
            //    and reads all 32 columns of a 16-row tile before writing it
            for (int rt = 0; rt < NPC / 16 / kBlkWaves; rt++) {
                const int row0 = (wv * (NPC / 16 / kBlkWaves) + rt) * 16;
                d4 d0 = {0.0, 0.0, 0.0, 0.0}, d1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < LOC / 4; kk++) {
                    const double av = Cs[(4 * kk + l4) * LDC + row0 + l16];
                    d0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Vs[4 * kk + l4][l16], d0, 0, 0, 0);
                    d1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Vs[4 * kk + l4][16 + l16], d1, 0, 0, 0);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    Cs[l16 * LDC + row0 + l4 + 4 * r] = d0[r];
                    Cs[(16 + l16) * LDC + row0 + l4 + 4 * r] = d1[r];
                }
            }
            __syncthreads();
            for (int e = tid; e < LOC * NPC; e += kBlkThreads) {
                const int l = e / NPC, i = e - l * NPC;
                const int col = (l < kBlk ? bp * kBlk + l : bq * kBlk + (l - kBlk));
                C[(int64_t)col * NPC + i] = Cs[l * LDC + i];
            }
            if (tid == 0 && s_rot) atomicExch(&ctrl[CTRL_FLAG + sweep % 3], 1);
            epoch++;
            if (!grid_barrier(ctrl, epoch * P)) {
                alive = false;
                break;
            }
        }
        if (!alive) break;
        sweeps++;
        if (atomicAdd(&ctrl[CTRL_FLAG + sweep % 3], 0) == 0) break;
    }
    if (w == 0 && tid == 0) ctrl[CTRL_SWEEPS] = alive ? sweeps : -1;
}

// sigma_k = |column k|, sorted descending (NaN everywhere after a timed-out run).
__global__ __launch_bounds__(1024) void k_jacobi_blk_finish(const double *C, int n, int npc, const int32_t *ctrl,
                                                            double *sigma)
{
    __shared__ double sv[512];
    const bool bad = ctrl[CTRL_SWEEPS] < 0;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        double acc = 0.0;
        for (int i = 0; i < npc; i++) acc = fma(C[(int64_t)k * npc + i], C[(int64_t)k * npc + i], acc);
        sv[k] = sqrt(acc);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const double v = sv[k];
        int rank = 0;
        for (int j = 0; j < n; j++) {
            const double u = sv[j];
            rank += (u > v) || (u == v && j < k);
        }
        sigma[rank] = bad ? __builtin_nan("") : ldexp(v, ctrl[CTRL_EXP]);
    }
}

template <int NPC>
hipError_t launch_blk(const double *R, int n, int64_t ldr, double *sigma, int max_sweeps, int32_t *ctrl,
                      double *C, hipStream_t s)
{
    const int64_t total = (int64_t)NPC * NPC;
    k_jacobi_blk_init<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(R, n, ldr, C, NPC, ctrl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_jacobi_blk<NPC><<<NPC / (2 * kBlk), kBlkThreads, 0, s>>>(C, n, max_sweeps, ctrl);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_jacobi_blk_finish<<<1, 1024, 0, s>>>(C, n, NPC, ctrl, sigma);
    return hipGetLastError();
}

}  // namespace

int64_t jacobi_scratch_doubles(int n)
{
    if (n <= 128) return 0;
    const int64_t npc = n <= 256 ? 256 : 512;
    return npc * npc;
}

hipError_t launch_jacobi(const double *R, int n, int64_t ldr, double *sigma, int max_sweeps,
                         int32_t *ctrl, double *scratch, hipStream_t s)
{
    if (n <= 0) return hipErrorInvalidValue;
    if (n <= 8) return launch_npc<8>(R, n, ldr, sigma, max_sweeps, ctrl, s);
    if (n <= 16) return launch_npc<16>(R, n, ldr, sigma, max_sweeps, ctrl, s);
    if (n <= 32) return launch_npc<32>(R, n, ldr, sigma, max_sweeps, ctrl, s);
    if (n <= 64) return launch_npc<64>(R, n, ldr, sigma, max_sweeps, ctrl, s);
    if (n <= 128) return launch_npc<128>(R, n, ldr, sigma, max_sweeps, ctrl, s);
    if (!scratch) return hipErrorInvalidValue;
    if (n <= 256) return launch_blk<256>(R, n, ldr, sigma, max_sweeps, ctrl, scratch, s);
    if (n <= 512) return launch_blk<512>(R, n, ldr, sigma, max_sweeps, ctrl, scratch, s);
    return hipErrorInvalidValue;
}

}  // namespace figaro

// ------------------------------------------------------------------ sigma via bidiagonalisation (n <= 128)
//
// The route of a dense SVD of R (Related Works: SVD through QR): Householder
// bidiagonalisation B = U^T R V (alternating a left reflector on column k and
// a right reflector on row k), then the singular values of the bidiagonal
// B = bidiag(d, e) as the positive eigenvalues of its Golub-Kahan tridiagonal
// (zero diagonal, off-diagonals d1, e1, d2, e2, ...), located by multisection
// on Sturm counts: the number of eigenvalues below x is the number of negative
// pivots of the LDL^T factorisation of T - x I.  Reflector conventions are the
// TSQR ones (beta = -sign(alpha) |(alpha, x)|, tau = 1 - alpha / beta).

namespace figaro {
namespace {

constexpr int kGkThreads = 256;   // load and scale; four waves bidiagonalise (NPC <= 64)
// Threads of the bidiagonalisation workgroup: eight waves at NPC = 128, four below.
template <int NPC>
__host__ __device__ constexpr int gk_threads() { return NPC == 128 ? 512 : kGkThreads; }
constexpr int kMsThreads = 256;   // multisection points per round (one workgroup per value)
constexpr int kMsRounds = 7;      // 257^7 > 2^55: the final interval is below 2^-53 of the bound

template <int NPC>
struct GkGeom {
    // row stride of A in LDS: even, so that rows are 16-byte aligned and a lane reading
    // its own row can use 128-bit reads; lane i then starts 4 i banks further, so 16
    // lanes cover the 64 banks (the fewest passes a 128-bit read of 64 lanes can take)
    static constexpr int LDA = NPC + 2;
};

// Reflector scalars for (alpha, s = |x|^2): tau, beta, scl = 1 / (alpha - beta); tau = 0 if s is 0.
__device__ inline void gk_reflector(double alpha, double s, double &tau, double &beta, double &scl)
{
    const double q = fma(alpha, alpha, s);
    tau = 0.0;
    beta = alpha;
    scl = 0.0;
    if (s > 0.0 && q >= DBL_MIN) {
        const double r = rsq_refined(q);
        const double sg = alpha >= 0.0 ? 1.0 : -1.0;
        const double nrm = q * r;
        beta = -sg * nrm;
        scl = rcp_refined(alpha + sg * nrm);
        tau = 1.0 - alpha * (-sg * r);
    }
}

__device__ inline double readlane_f64(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// Sum over an aligned group of G lanes (G a power of two <= 16) with DPP moves.
template <int G>
__device__ inline double dpp_group_sum(double v)
{
    if constexpr (G >= 2) v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    if constexpr (G >= 4) v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    if constexpr (G >= 8) v += dpp_f64<0x141>(v);  // row_half_mirror
    if constexpr (G >= 16) v += dpp_f64<0x140>(v); // row_mirror
    return v;
}

// Sum over the whole wave, the same value in every lane: rows of 16 by DPP, then the
// four row sums read back by lane.
__device__ inline double wave_sum(double v)
{
    v = dpp_group_sum<16>(v);
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// The same bidiagonalisation by the four waves of the workgroup (NPC <= 64).  Every wave
// forms the reflector of a half-step itself, from the column (left) or row (right) it
// reads from LDS, and applies it to its quarter of the rows (left: lane = column) or of
// the columns (right: lane = row), entries [w RW, (w + 1) RW): the quarter is loaded
// right after the barrier, the reflector entries of the quarter come from lane reads,
// the per-lane partial dot products meet in LDS (one barrier), the wave updates its
// quarter, and a second barrier publishes the matrix for the next half-step.
template <int NPC>
__device__ void gk_bidiag_wg(double *A, double (*red)[64], double *dd, double *ee, int n, int lane, int wv)
{
    constexpr int LDA = GkGeom<NPC>::LDA, RW = NPC / 4;
    const int w = __builtin_amdgcn_readfirstlane(wv);
    const int e0 = w * RW;                      // first entry of this wave's quarter
    const int ln = lane < NPC ? lane : NPC - 1;  // this lane's column (row) of A, clamped
    for (int k = 0; k < n; k++) {
        // ---- left reflector from column k (rows k..n-1), applied to the columns j > k
        {
            double x[RW];  // A[e0 + r][lane]
#pragma unroll
            for (int r = 0; r < RW; r++) x[r] = A[(e0 + r) * LDA + ln];
            const double a = A[ln * LDA + k];
            const double s = wave_sum(lane > k && lane < n ? a * a : 0.0);
            const double alpha = readlane_f64(a, k);
            double tau, beta, scl;
            gk_reflector(alpha, s, tau, beta, scl);
            const double v = lane == k ? 1.0 : (lane > k && lane < n ? a * scl : 0.0);
            double ve[RW], p[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int r = 0; r < RW; r++) {
                ve[r] = readlane_f64(v, e0 + r);
                p[r & 3] = fma(ve[r], x[r], p[r & 3]);
            }
            red[w][lane] = (p[0] + p[1]) + (p[2] + p[3]);
            __syncthreads();
            const double t = ((red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane])) * tau;
            if (lane > k && lane < n && e0 + RW > k) {
#pragma unroll
                for (int r = 0; r < RW; r++) A[(e0 + r) * LDA + lane] = fma(-t, ve[r], x[r]);
            }
            if (lane == 0 && w == 0) dd[k] = beta;
            __syncthreads();
        }
        if (k + 1 >= n) break;
        // ---- right reflector from row k (columns k+1..n-1), applied to the rows i > k
        {
            double x[RW];  // A[lane][e0 + r]
#pragma unroll
            for (int r = 0; r < RW; r++) x[r] = A[ln * LDA + e0 + r];
            const double rk = A[k * LDA + ln];
            const double s = wave_sum(lane > k + 1 && lane < n ? rk * rk : 0.0);
            const double alpha = readlane_f64(rk, k + 1);
            double tau, beta, scl;
            gk_reflector(alpha, s, tau, beta, scl);
            const double v = lane == k + 1 ? 1.0 : (lane > k + 1 && lane < n ? rk * scl : 0.0);
            double ve[RW], p[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int r = 0; r < RW; r++) {
                ve[r] = readlane_f64(v, e0 + r);
                p[r & 3] = fma(ve[r], x[r], p[r & 3]);
            }
            red[w][lane] = (p[0] + p[1]) + (p[2] + p[3]);
            __syncthreads();
            const double t = ((red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane])) * tau;
            if (lane > k && lane < n && e0 + RW > k + 1) {
#pragma unroll
                for (int r = 0; r < RW; r++) A[lane * LDA + e0 + r] = fma(-t, ve[r], x[r]);
            }
            if (lane == 0 && w == 0) ee[k] = beta;
            __syncthreads();
        }
    }
}

// The same by eight waves at NPC = 128: every lane owns two columns (left half-step) or
// two rows (right half-step), c = lane + 64 u, and each wave an eighth of the other index
// (16 entries in registers); the partial dot products of the two columns (rows) meet in
// LDS as above.
template <int NPC>
__device__ void gk_bidiag_wg2(double *A, double (*red)[NPC], double *dd, double *ee, int n, int lane, int wv)
{
    static_assert(NPC == 128, "two columns per lane");
    constexpr int W = gk_threads<NPC>() / 64;
    constexpr int LDA = GkGeom<NPC>::LDA, RW = NPC / W;
    const int w = __builtin_amdgcn_readfirstlane(wv);
    const int e0 = w * RW;          // first entry of this wave's share
    const int vsel = e0 / 64;       // the reflector entries e0 .. e0 + RW - 1 sit in v[vsel]
    const int voff = e0 % 64;
    for (int k = 0; k < n; k++) {
        // ---- left reflector from column k (rows k..n-1), applied to the columns j > k
        {
            double x[2][RW];  // A[e0 + r][lane + 64 u]
#pragma unroll
            for (int u = 0; u < 2; u++)
#pragma unroll
                for (int r = 0; r < RW; r++) x[u][r] = A[(e0 + r) * LDA + lane + 64 * u];
            double a[2], v[2];
            double ss = 0.0;
#pragma unroll
            for (int u = 0; u < 2; u++) {
                const int i = lane + 64 * u;
                a[u] = A[i * LDA + k];
                ss = fma(i > k && i < n ? a[u] : 0.0, a[u], ss);
            }
            const double s = wave_sum(ss);
            const double alpha = readlane_f64(k < 64 ? a[0] : a[1], k & 63);
            double tau, beta, scl;
            gk_reflector(alpha, s, tau, beta, scl);
#pragma unroll
            for (int u = 0; u < 2; u++) {
                const int i = lane + 64 * u;
                v[u] = i == k ? 1.0 : (i > k && i < n ? a[u] * scl : 0.0);
            }
            const double vq = vsel ? v[1] : v[0];
            double ve[RW], p[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
            for (int r = 0; r < RW; r++) {
                ve[r] = readlane_f64(vq, voff + r);
#pragma unroll
                for (int u = 0; u < 2; u++) p[u][r & 1] = fma(ve[r], x[u][r], p[u][r & 1]);
            }
#pragma unroll
            for (int u = 0; u < 2; u++) red[w][lane + 64 * u] = p[u][0] + p[u][1];
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 2; u++) {
                const int j = lane + 64 * u;
                double t = 0.0;
#pragma unroll
                for (int q = 0; q < W; q += 4) t += (red[q][j] + red[q + 1][j]) + (red[q + 2][j] + red[q + 3][j]);
                t *= tau;
                if (j > k && j < n && e0 + RW > k) {
#pragma unroll
                    for (int r = 0; r < RW; r++) A[(e0 + r) * LDA + j] = fma(-t, ve[r], x[u][r]);
                }
            }
            if (lane == 0 && w == 0) dd[k] = beta;
            __syncthreads();
        }
        if (k + 1 >= n) break;
        // ---- right reflector from row k (columns k+1..n-1), applied to the rows i > k
        {
            double x[2][RW];  // A[lane + 64 u][e0 + r]
#pragma unroll
            for (int u = 0; u < 2; u++)
#pragma unroll
                for (int r = 0; r < RW; r++) x[u][r] = A[(lane + 64 * u) * LDA + e0 + r];
            double rk[2], v[2];
            double ss = 0.0;
#pragma unroll
            for (int u = 0; u < 2; u++) {
                const int j = lane + 64 * u;
                rk[u] = A[k * LDA + j];
                ss = fma(j > k + 1 && j < n ? rk[u] : 0.0, rk[u], ss);
            }
            const double s = wave_sum(ss);
            const double alpha = readlane_f64(k + 1 < 64 ? rk[0] : rk[1], (k + 1) & 63);
            double tau, beta, scl;
            gk_reflector(alpha, s, tau, beta, scl);
#pragma unroll
            for (int u = 0; u < 2; u++) {
                const int j = lane + 64 * u;
                v[u] = j == k + 1 ? 1.0 : (j > k + 1 && j < n ? rk[u] * scl : 0.0);
            }
            const double vq = vsel ? v[1] : v[0];
            double ve[RW], p[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
            for (int r = 0; r < RW; r++) {
                ve[r] = readlane_f64(vq, voff + r);
#pragma unroll
                for (int u = 0; u < 2; u++) p[u][r & 1] = fma(ve[r], x[u][r], p[u][r & 1]);
            }
#pragma unroll
            for (int u = 0; u < 2; u++) red[w][lane + 64 * u] = p[u][0] + p[u][1];
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 2; u++) {
                const int i = lane + 64 * u;
                double t = 0.0;
#pragma unroll
                for (int q = 0; q < W; q += 4) t += (red[q][i] + red[q + 1][i]) + (red[q + 2][i] + red[q + 3][i]);
                t *= tau;
                if (i > k && i < n && e0 + RW > k + 1) {
#pragma unroll
                    for (int r = 0; r < RW; r++) A[i * LDA + e0 + r] = fma(-t, ve[r], x[u][r]);
                }
            }
            if (lane == 0 && w == 0) ee[k] = beta;
            __syncthreads();
        }
    }
}

template <int NPC>
__device__ __forceinline__ void sigma_gk_body(const double *R, int n, int64_t ldr, double *msin, int32_t *ctrl)
{
    using Gm = GkGeom<NPC>;
    constexpr int LDA = Gm::LDA;
    __shared__ double A[NPC * LDA];
    __shared__ double red[gk_threads<NPC>() / 64][NPC > 64 ? NPC : 64];
    __shared__ double dd[NPC], ee[NPC];
    __shared__ double sc[2];
    __shared__ int s_exp;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (ctrl && tid < CTRL_WORDS) ctrl[tid] = 0;  // no sweeps: this route does not iterate
    if (tid == 0) s_exp = INT_MIN;
    staged_copy<16, double>(
        NPC * NPC, tid, gk_threads<NPC>(),
        [&](int e) {
            const int i = e / NPC, j = e - i * NPC;
            return R[(int64_t)(i < n ? i : n - 1) * ldr + (j < n ? j : n - 1)];
        },
        [&](int e, double v) {
            const int i = e / NPC, j = e - i * NPC;
            A[i * LDA + j] = (i < n && j < n) ? v : 0.0;
        });
    __syncthreads();
    // Scale by a power of two so that the largest |entry| lies in [1, 2) (exact): the
    // reflector norms and the recurrence below stay in range.
    {
        double m = 0.0;
        for (int e = tid; e < NPC * NPC; e += gk_threads<NPC>()) m = fmax(m, fabs(A[(e / NPC) * LDA + e % NPC]));
        if (m > 0.0) atomicMax(&s_exp, ilogb(m));
    }
    __syncthreads();
    const int ex0 = s_exp == INT_MIN ? 0 : s_exp;
    for (int e = tid; e < NPC * NPC; e += gk_threads<NPC>()) {
        double &x = A[(e / NPC) * LDA + e % NPC];
        x = ldexp(x, -ex0);
    }
    __syncthreads();
    if constexpr (NPC <= 64) {
        gk_bidiag_wg<NPC>(A, red, dd, ee, n, lane, wv);
    } else {
        gk_bidiag_wg2<NPC>(A, red, dd, ee, n, lane, wv);
    }
    __syncthreads();
    // ---- inputs of the multisection: the Golub-Kahan tridiagonal T (zero diagonal,
    // off-diagonals d1, e1, d2, ...) scaled once more so that its Gershgorin bound lies in
    // [1, 2); msin = {bound, total binary exponent, squared off-diagonals}.
    if (tid == 0) {
        double h = 0.0;
        for (int i = 0; i < n; i++) {
            const double a = fabs(dd[i]) + (i + 1 < n ? fabs(ee[i]) : 0.0) + (i > 0 ? fabs(ee[i - 1]) : 0.0);
            h = fmax(h, a);
        }
        const int ex = h > 0.0 ? ilogb(h) : 0;
        sc[0] = (double)ex;
        msin[0] = ldexp(h, -ex);
        msin[1] = (double)(ex + ex0);
    }
    __syncthreads();
    const int ex = (int)sc[0];
    for (int i = tid; i < 2 * n - 1; i += gk_threads<NPC>()) {
        const double b = ldexp((i & 1) ? ee[i >> 1] : dd[i >> 1], -ex);
        msin[2 + i] = b * b;
    }
}

template <int NPC>
__global__ __launch_bounds__(gk_threads<NPC>()) void k_sigma_gk(const double *R, int n, int64_t ldr, double *msin, int32_t *ctrl)
{
    sigma_gk_body<NPC>(R, n, ldr, msin, ctrl);
}

// Many independent problems of one width class: workgroup b takes entry b of tab (4 int64
// each: element offset of its n x n R, offset of its sigma, n, offset of its msin).
template <int NPC>
__global__ __launch_bounds__(gk_threads<NPC>()) void k_sigma_gk_batch(const double *R, const int64_t *tab, double *msin)
{
    const int64_t *e = tab + 4 * (int64_t)blockIdx.x;
    const int n = (int)e[2];
    sigma_gk_body<NPC>(R + e[0], n, n, msin + e[3], nullptr);
}

// One step of the Sturm sequence: p2 = -x p1 - b p0, then DBL_MIN with the sign opposite
// to p1 added.  An exact zero becomes that tiny value (a zero term counts as a sign
// change: a zero pivot taken negative); any term of magnitude above 2^-1020 is unchanged
// by the addition, and the rescaling every 16 steps keeps the nonzero terms far above
// it.  cnt counts the sign changes from the sign bits.
__device__ inline void sturm_step(double x, double b, double &p0, double &p1, int &cnt)
{
    const int h1 = __double2hiint(p1);
    const double bias = __hiloint2double((h1 & (int)0x80000000) ^ (int)0x80100000, 0);  // -sign(p1) DBL_MIN
    const double p2 = fma(-x, p1, -b * p0) + bias;
    cnt += (int)(((unsigned)(__double2hiint(p2) ^ h1)) >> 31);
    p0 = p1;
    p1 = p2;
}

// Number of eigenvalues of the Golub-Kahan tridiagonal (zero diagonal, squared
// off-diagonals bb[0..m-1]) below x: the sign changes of its characteristic sequence
// p_0 = 1, p_1 = -x, p_i = -x p_{i-1} - bb_{i-2} p_{i-2}.  The pair (p_{i-1}, p_i) is
// rescaled by a power of two every 16 steps, which keeps it in range and changes no sign.
__device__ inline int gk_sturm_count(const double *bb, int m, double x)
{
    double p0 = 1.0, p1 = -x;
    int cnt = (int)(((unsigned)__double2hiint(p1)) >> 31);  // signs are read from the sign bits throughout
    // chunks of 16 steps with their coefficients loaded up front (the recurrence does not
    // wait on LDS; bb holds whole chunks, entries past m unused): full chunks, then the
    // last one step by step under a uniform condition
    for (int i0 = 0; i0 < m; i0 += 16) {
        double b[16];
#pragma unroll
        for (int u = 0; u < 16; u++) b[u] = bb[i0 + u];
        if (i0 + 16 <= m) {
#pragma unroll
            for (int u = 0; u < 16; u++) sturm_step(x, b[u], p0, p1, cnt);
        } else {
#pragma unroll
            for (int u = 0; u < 16; u++)
                if (i0 + u < m) sturm_step(x, b[u], p0, p1, cnt);
        }
        const int e2 = ilogb(fmax(fabs(p0), fabs(p1)));
        p0 = ldexp(p0, -e2);
        p1 = ldexp(p1, -e2);
    }
    return cnt;
}

// Multisection for the singular values of the bidiagonal: workgroup k locates sigma_k
// (the k-th largest), which lies in [0, bound].  sigma_k < x exactly when at least 2n - k
// eigenvalues of T lie below x.  Each round evaluates the count at kMsThreads points
// evenly inside the current interval and keeps the gap between the last point whose count
// is below 2n - k and the first point whose count is not.
__device__ __forceinline__ void sigma_msect_body(const double *msin, int n, int k, double *sigma)
{
    constexpr int NW = kMsThreads / 64;
    __shared__ double bb[256];  // 2n - 1 <= 255 coefficients, read in chunks of 16
    __shared__ int s_lo[2][NW], s_up[2][NW];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = 2 * n - 1;
    for (int i = tid; i < m; i += kMsThreads) bb[i] = msin[2 + i];
    const double bound = msin[0];
    const int ex = (int)msin[1];
    __syncthreads();
    const int target = 2 * n - k;
    const double step = 1.0 / (double)(kMsThreads + 1);
    double lo = 0.0, up = bound;
    for (int it = 0; it < kMsRounds; it++) {
        const double w = up - lo;
        const double x = lo + w * ((double)(tid + 1) * step);
        const bool below = gk_sturm_count(bb, m, x) < target;
        const unsigned long long mask = __ballot(below);
        if (lane == 0) {
            // last point of this wave below the target, first one not below
            s_lo[it & 1][wv] = mask ? wv * 64 + 63 - __builtin_clzll(mask) : -1;
            s_up[it & 1][wv] = ~mask ? wv * 64 + __builtin_ctzll(~mask) : kMsThreads;
        }
        __syncthreads();
        int ilo = -1, iup = kMsThreads;
#pragma unroll
        for (int q = 0; q < NW; q++) {
            ilo = max(ilo, s_lo[it & 1][q]);
            iup = min(iup, s_up[it & 1][q]);
        }
        // every thread recomputes the two points exactly as their lanes did
        const double xlo = ilo >= 0 ? lo + w * ((double)(ilo + 1) * step) : lo;
        const double xup = iup < kMsThreads ? lo + w * ((double)(iup + 1) * step) : up;
        lo = xlo;
        up = xup;
    }
    if (tid == 0) sigma[k] = ldexp(0.5 * (lo + up), ex);
}

__global__ __launch_bounds__(kMsThreads) void k_sigma_msect(const double *msin, int n, double *sigma)
{
    sigma_msect_body(msin, n, blockIdx.x, sigma);
}

// Multisection by lane groups, for batches: G lanes locate one value with G points per
// round (a wave holds 64 / G values; a workgroup 4 waves of one entry).  Fewer points per
// round need more rounds, (G + 1)^rounds > 2^55 as above, but far fewer Sturm counts per
// value (G = 16: 14 x 16 instead of 7 x 256), and no workgroup barrier inside the rounds.
template <int G>
struct MsWave {
    static constexpr int VPW = 64 / G;                  // values per wave
    static constexpr int VPB = 4 * VPW;                 // values per workgroup
    static constexpr int ROUNDS = G == 16 ? 14 : G == 8 ? 19 : G == 4 ? 24 : 10;
};

template <int G>
__device__ __forceinline__ void sigma_msect_wave_body(const double *msin, int n, int k0, double *sigma)
{
    static_assert(G == 4 || G == 8 || G == 16 || G == 64, "lane group");
    __shared__ double bb[256];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = 2 * n - 1;
    for (int i = tid; i < m; i += 256) bb[i] = msin[2 + i];
    const double bound = msin[0];
    const int ex = (int)msin[1];
    __syncthreads();
    const int grp = lane / G, idx = lane % G;
    const int k = k0 + wv * MsWave<G>::VPW + grp;
    const int target = 2 * n - k;
    const double step = 1.0 / (double)(G + 1);
    const unsigned long long gmask = G == 64 ? ~0ull : ((1ull << G) - 1);
    double lo = 0.0, up = bound;
    for (int it = 0; it < MsWave<G>::ROUNDS; it++) {
        const double w = up - lo;
        const double x = lo + w * ((double)(idx + 1) * step);
        const bool below = gk_sturm_count(bb, m, x) < target;
        const unsigned long long mk = (__ballot(below) >> (grp * G)) & gmask;
        // last point of the group below the target, first one not below
        const int ilo = mk ? 63 - __builtin_clzll(mk) : -1;
        const unsigned long long nm = ~mk & gmask;
        const int iup = nm ? __builtin_ctzll(nm) : G;
        const double xlo = ilo >= 0 ? lo + w * ((double)(ilo + 1) * step) : lo;
        const double xup = iup < G ? lo + w * ((double)(iup + 1) * step) : up;
        lo = xlo;
        up = xup;
    }
    if (idx == 0 && k < n) sigma[k] = ldexp(0.5 * (lo + up), ex);
}

// Workgroup (b, e) locates values [b VPB, (b + 1) VPB) of entry e of tab (entries as
// k_sigma_gk_batch); workgroups past the entry's width leave at once.
template <int G>
__global__ __launch_bounds__(256) void k_sigma_msect_wave_batch(const int64_t *tab, const double *msin,
                                                                double *sigma)
{
    const int64_t *e = tab + 4 * (int64_t)blockIdx.y;
    const int n = (int)e[2], k0 = blockIdx.x * MsWave<G>::VPB;
    if (k0 >= n) return;
    sigma_msect_wave_body<G>(msin + e[3], n, k0, sigma + e[1]);
}

// ------------------------------------------------------------------ dqds
//
// The squareroot-free route for singular values alone (Related Works: dqds).  The
// bidiagonal B (diagonal d, superdiagonal e) left by the bidiagonalisation is held as
// q_i = d_i^2 and e_i = e_i^2 (the multisection inputs: the Golub-Kahan off-diagonals
// squared, d_1^2, e_1^2, d_2^2, ...).  One differential qd transform with shift tau:
//     d = q_1 - tau;  for i < N:  qh_i = d + e_i,  t = q_{i+1} / qh_i,  eh_i = e_i t,
//                                 d = d t - tau;  qh_N = d,
// maps the pair to that of B^T B - tau I with every quantity positive while tau is below
// its smallest eigenvalue.  Transforms repeat until the last e is negligible; then
// q_N + (the shifts so far) is an eigenvalue of B^T B and the bottom row is deflated.
// Shifts: half the smallest d of the previous transform; a transform that would turn a
// quantity negative is undone and repeated with tau = 0, which cannot fail.  A zero e
// (split) passes d on unchanged.  One thread per problem (the transforms are a serial
// recurrence); sigma = 2^ex sqrt(lambda), sorted descending.
constexpr int kDqdsMaxN = 128;

// qs, es: room for a copy of q and e (LDS), to undo a failed transform.
__device__ void dqds_serial(double *q, double *e, int n, double scale2, double *lam, double *qs, double *es)
{
    const double eps = 0x1p-53;
    const double tiny = eps * eps * scale2;  // squares below this are zero at the working precision
    int N = n;
    double S = 0.0;     // shifts applied to the active rows so far
    double tau = 0.0;
    int iters = 0;
    const int max_iters = 64 * n + 64;
    while (N > 0) {
        if (N == 1) {
            lam[0] = q[0] + S;
            break;
        }
        const double en = e[N - 2];
        if (en <= eps * (q[N - 1] + S) || en <= tiny || iters >= max_iters) {
            lam[N - 1] = q[N - 1] + S;
            N--;
            tau = 0.0;
            continue;
        }
        iters++;
        for (int i = 0; i < N; i++) qs[i] = q[i];
        for (int i = 0; i < N - 1; i++) es[i] = e[i];
        bool ok;
        double dmin;
        for (;;) {
            ok = true;
            double d = q[0] - tau;
            dmin = d;
            if (d < 0.0) ok = false;
            for (int i = 0; ok && i < N - 1; i++) {
                if (e[i] == 0.0) {
                    q[i] = d;
                    d = q[i + 1] - tau;
                } else {
                    const double qh = d + e[i];
                    if (!(qh > 0.0)) {
                        ok = false;
                        break;
                    }
                    const double t = q[i + 1] / qh;
                    e[i] = e[i] * t;
                    q[i] = qh;
                    d = d * t - tau;
                }
                if (d < 0.0) ok = false;
                dmin = fmin(dmin, d);
            }
            if (ok) {
                q[N - 1] = d;
                break;
            }
            // undo and repeat without a shift
            for (int i = 0; i < N; i++) q[i] = qs[i];
            for (int i = 0; i < N - 1; i++) e[i] = es[i];
            if (tau == 0.0) {  // cannot happen in exact arithmetic; take the values as they are
                dmin = 0.0;
                break;
            }
            tau = 0.0;
        }
        S += tau;
        tau = 0.5 * fmax(dmin, 0.0);
    }
}

__device__ __forceinline__ void sigma_dqds_body(const double *msin, int n, double *sigma)
{
    __shared__ double q[kDqdsMaxN], e[kDqdsMaxN], lam[kDqdsMaxN], qs[kDqdsMaxN], es[kDqdsMaxN];
    const int tid = threadIdx.x;
    for (int i = tid; i < n; i += blockDim.x) {
        q[i] = msin[2 + 2 * i];
        e[i] = i + 1 < n ? msin[3 + 2 * i] : 0.0;
    }
    __syncthreads();
    const double bound = msin[0];
    const int ex = (int)msin[1];
    if (tid == 0) dqds_serial(q, e, n, bound * bound, lam, qs, es);
    __syncthreads();
    for (int k = tid; k < n; k += blockDim.x) {
        const double v = lam[k];
        int rank = 0;
        for (int j = 0; j < n; j++) rank += (lam[j] > v) || (lam[j] == v && j < k);
        sigma[rank] = ldexp(sqrt(fmax(v, 0.0)), ex);
    }
}

__global__ __launch_bounds__(64) void k_sigma_dqds(const double *msin, int n, double *sigma)
{
    sigma_dqds_body(msin, n, sigma);
}

// Batched: workgroup b takes entry b of tab (entries as k_sigma_gk_batch).
__global__ __launch_bounds__(64) void k_sigma_dqds_batch(const int64_t *tab, const double *msin, double *sigma)
{
    const int64_t *e = tab + 4 * (int64_t)blockIdx.x;
    sigma_dqds_body(msin + e[3], (int)e[2], sigma + e[1]);
}

template <int NPC>
hipError_t launch_gk(const double *R, int n, int64_t ldr, int32_t *ctrl, double *msin, hipStream_t s)
{
    k_sigma_gk<NPC><<<1, gk_threads<NPC>(), 0, s>>>(R, n, ldr, msin, ctrl);
    return hipGetLastError();
}

}  // namespace

int64_t svd_v_scratch_doubles(int n)
{
    const int npc = n <= 8 ? 8 : n <= 16 ? 16 : n <= 32 ? 32 : n <= 64 ? 64 : 128;
    return (int64_t)npc * npc;
}

hipError_t launch_svd_v(const double *R, int n, int64_t ldr, double *sigma, double *V, int64_t ldv, int max_sweeps,
                        int32_t *ctrl, double *scratch, hipStream_t s)
{
    if (n < 1 || n > 128) return hipErrorInvalidValue;
    if (n <= 8) return launch_v_npc<8>(R, n, ldr, sigma, max_sweeps, ctrl, scratch, V, ldv, s);
    if (n <= 16) return launch_v_npc<16>(R, n, ldr, sigma, max_sweeps, ctrl, scratch, V, ldv, s);
    if (n <= 32) return launch_v_npc<32>(R, n, ldr, sigma, max_sweeps, ctrl, scratch, V, ldv, s);
    if (n <= 64) return launch_v_npc<64>(R, n, ldr, sigma, max_sweeps, ctrl, scratch, V, ldv, s);
    return launch_v_npc<128>(R, n, ldr, sigma, max_sweeps, ctrl, scratch, V, ldv, s);
}

int64_t sigma_bidiag_scratch_doubles(int n) { return n <= 128 ? 2 * (int64_t)n + 2 : 0; }

hipError_t launch_sigma_bidiag(const double *R, int n, int64_t ldr, int32_t *ctrl, double *msin, hipStream_t s)
{
    if (n <= 0 || !msin) return hipErrorInvalidValue;
    if (n <= 8) return launch_gk<8>(R, n, ldr, ctrl, msin, s);
    if (n <= 16) return launch_gk<16>(R, n, ldr, ctrl, msin, s);
    if (n <= 32) return launch_gk<32>(R, n, ldr, ctrl, msin, s);
    if (n <= 64) return launch_gk<64>(R, n, ldr, ctrl, msin, s);
    if (n <= 128) return launch_gk<128>(R, n, ldr, ctrl, msin, s);
    return hipErrorInvalidValue;
}

hipError_t launch_sigma_dqds(const double *msin, int n, double *sigma, hipStream_t s)
{
    if (n <= 0 || n > kDqdsMaxN) return hipErrorInvalidValue;
    k_sigma_dqds<<<1, 64, 0, s>>>(msin, n, sigma);
    return hipGetLastError();
}

hipError_t launch_sigma_msect(const double *msin, int n, double *sigma, hipStream_t s)
{
    if (n <= 0 || n > 128 || !msin) return hipErrorInvalidValue;
    k_sigma_msect<<<n, kMsThreads, 0, s>>>(msin, n, sigma);
    return hipGetLastError();
}

int sigma_width_class(int n)
{
    int npc = 8;
    while (npc < n) npc *= 2;
    return npc <= 128 ? npc : 0;
}

hipError_t launch_sigma_batch(int npc, const double *R, double *sigma, const int64_t *tab, int count, double *msin,
                              hipStream_t s, int dqds)
{
    if (count <= 0) return hipSuccess;
    switch (npc) {
    case 8: k_sigma_gk_batch<8><<<count, gk_threads<8>(), 0, s>>>(R, tab, msin); break;
    case 16: k_sigma_gk_batch<16><<<count, gk_threads<16>(), 0, s>>>(R, tab, msin); break;
    case 32: k_sigma_gk_batch<32><<<count, gk_threads<32>(), 0, s>>>(R, tab, msin); break;
    case 64: k_sigma_gk_batch<64><<<count, gk_threads<64>(), 0, s>>>(R, tab, msin); break;
    case 128: k_sigma_gk_batch<128><<<count, gk_threads<128>(), 0, s>>>(R, tab, msin); break;
    default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (dqds) k_sigma_dqds_batch<<<count, 64, 0, s>>>(tab, msin, sigma);
    else if (npc == 128) {
        // the widest class holds the most values, and its launch is bound by the issue rate
        // of the Sturm counts: 4 lanes per value (24 rounds, 96 counts per value) beat 16
        // (14 rounds, 224 counts) there, while the narrower classes, with fewer values, are
        // bound by the rounds' latency and keep 16 (measured on the 256-instance batch)
        constexpr int G = 4;
        const unsigned nb = (unsigned)((npc + MsWave<G>::VPB - 1) / MsWave<G>::VPB);
        k_sigma_msect_wave_batch<G><<<dim3(nb, count), 256, 0, s>>>(tab, msin, sigma);
    } else {
        constexpr int G = 16;
        const unsigned nb = (unsigned)((npc + MsWave<G>::VPB - 1) / MsWave<G>::VPB);
        k_sigma_msect_wave_batch<G><<<dim3(nb, count), 256, 0, s>>>(tab, msin, sigma);
    }
    return hipGetLastError();
}

}  // namespace figaro
