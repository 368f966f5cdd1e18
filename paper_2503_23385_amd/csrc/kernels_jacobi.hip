// Singular values of R by one-sided (Hestenes) Jacobi in FP64.
//
// The singular values of the join matrix equal those of R (Related Works:
// SVD through QR); the paper obtains them with a dense SVD of R.  Here one
// workgroup keeps R's columns in LDS and orthogonalises column pairs with
// plane rotations until every pair satisfies |c_p . c_q| <= n 2^-53 |c_p||c_q|.
// Pairs are visited in a round-robin (circle) order: each of the n-1 steps of
// a sweep rotates n/2 disjoint pairs in parallel, so a sweep still meets
// every pair once.  For a pair with alpha = |c_p|^2, beta = |c_q|^2,
// gamma = c_p . c_q:
//     zeta = (beta - alpha) / (2 gamma),  t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
//     c = 1 / sqrt(1 + t^2),  s = c t,   (c_p, c_q) <- (c c_p - s c_q, s c_p + c c_q).
// sigma_k = |c_k| after convergence, sorted descending.
//
// Eight lanes share a pair and keep its two columns in registers for the
// whole step (one batch of LDS loads, one of stores); the three dot products
// are reduced with DPP moves inside the lane octet; one workgroup barrier
// separates the steps.  The width is a template parameter so every loop over
// rows is unrolled.
#include "common.h"

namespace figaro {
namespace {

constexpr int kLanesPerPair = 8;

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

// Sum over the 8-lane group (lanes 8g..8g+7) with DPP: xor 1, xor 2, then the
// mirror of the half-row (lane i <-> 7 - i), which swaps the two quads.
template <int CTRL>
__device__ inline double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ inline double octet_sum(double v)
{
    v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    return v;
}

// NPC: padded (even, power of two) column count; columns n..NPC-1 are zero.
template <int NPC>
__global__ __launch_bounds__(NPC * kLanesPerPair / 2 < 64 ? 64 : NPC * kLanesPerPair / 2)
void k_jacobi_lds(const double *R, int n, int64_t ldr, double *sigma, int max_sweeps,
                  int32_t *sweeps_out)
{
    constexpr int RPL = NPC / kLanesPerPair;  // rows per lane
    constexpr int PAIRS = NPC / 2;
    __shared__ double C[NPC * NPC];  // column k at C[k * NPC]
    __shared__ double sv[NPC];
    __shared__ int s_rot;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    for (int e = tid; e < NPC * NPC; e += nthr) {
        const int k = e / NPC, i = e - k * NPC;
        C[e] = (k < n && i < n) ? R[(int64_t)i * ldr + k] : 0.0;
    }
    const int pair = tid / kLanesPerPair, sub = tid % kLanesPerPair;
    const bool active = pair < PAIRS;
    const double tol2 = ((double)n * 0x1p-53) * ((double)n * 0x1p-53);
    constexpr int M = NPC - 1;
    int sweeps = 0;
    __syncthreads();
    for (int sweep = 0; sweep < max_sweeps; sweep++) {
        if (tid == 0) s_rot = 0;
        __syncthreads();
        for (int step = 0; step < M; step++) {
            int p = 0, q = 0;
            if (pair == 0) {
                p = step;
                q = NPC - 1;
            } else if (active) {
                p = (step + pair) % M;
                q = (step - pair + M) % M;
            }
            if (p > q) { const int t = p; p = q; q = t; }
            double *cp = C + p * NPC + sub, *cq = C + q * NPC + sub;
            double xp[RPL], xq[RPL];
#pragma unroll
            for (int r = 0; r < RPL; r++) {
                xp[r] = active ? cp[r * kLanesPerPair] : 0.0;
                xq[r] = active ? cq[r * kLanesPerPair] : 0.0;
            }
            double a = 0.0, b = 0.0, g = 0.0;
#pragma unroll
            for (int r = 0; r < RPL; r++) {
                a = fma(xp[r], xp[r], a);
                b = fma(xq[r], xq[r], b);
                g = fma(xp[r], xq[r], g);
            }
            a = octet_sum(a);
            b = octet_sum(b);
            g = octet_sum(g);
            if (active && g * g > tol2 * a * b) {
                const double zeta = (b - a) * rcp_refined(2.0 * g);
                double t;
                if (fabs(zeta) > 1e150) {
                    t = 0.5 * rcp_refined(zeta);  // sign(zeta) / (2 |zeta|): 1 + zeta^2 would overflow
                } else {
                    const double qq = fma(zeta, zeta, 1.0);
                    const double sq = qq * rsq_refined(qq);  // sqrt(1 + zeta^2)
                    t = (zeta >= 0.0 ? 1.0 : -1.0) * rcp_refined(fabs(zeta) + sq);
                }
                const double c = rsq_refined(fma(t, t, 1.0));
                const double s = c * t;
#pragma unroll
                for (int r = 0; r < RPL; r++) {
                    cp[r * kLanesPerPair] = c * xp[r] - s * xq[r];
                    cq[r * kLanesPerPair] = s * xp[r] + c * xq[r];
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
        for (int i = 0; i < NPC; i++) acc += C[k * NPC + i] * C[k * NPC + i];
        sv[k] = sqrt(acc);
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
    }
    if (tid == 0 && sweeps_out) *sweeps_out = sweeps;
}

template <int NPC>
hipError_t launch_npc(const double *R, int n, int64_t ldr, double *sigma, int max_sweeps,
                      int32_t *sweeps_out, hipStream_t s)
{
    int threads = NPC * kLanesPerPair / 2;
    if (threads < 64) threads = 64;
    k_jacobi_lds<NPC><<<1, threads, 0, s>>>(R, n, ldr, sigma, max_sweeps, sweeps_out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_jacobi(const double *R, int n, int64_t ldr, double *sigma, int max_sweeps,
                         int32_t *sweeps_out, hipStream_t s)
{
    if (n <= 0) return hipErrorInvalidValue;
    if (n <= 8) return launch_npc<8>(R, n, ldr, sigma, max_sweeps, sweeps_out, s);
    if (n <= 16) return launch_npc<16>(R, n, ldr, sigma, max_sweeps, sweeps_out, s);
    if (n <= 32) return launch_npc<32>(R, n, ldr, sigma, max_sweeps, sweeps_out, s);
    if (n <= 64) return launch_npc<64>(R, n, ldr, sigma, max_sweeps, sweeps_out, s);
    if (n <= 128) return launch_npc<128>(R, n, ldr, sigma, max_sweeps, sweeps_out, s);
    return hipErrorInvalidValue;
}

}  // namespace figaro
