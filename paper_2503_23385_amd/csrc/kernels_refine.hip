// One FP64 refinement sweep of an approximate R (the FP32 form's result).
//
// R is the Cholesky factor of J^T J (Section 1, Applications).  Without
// forming J, the Gram matrix has a closed form per key group g:
//     J^T J = sum_g [ m2_g A_g^T A_g ,  a_g b_g^T ;  b_g a_g^T ,  m1_g B_g^T B_g ],
// with a_g, b_g the column sums of the group's rows.  Given the approximate
// R~, the sweep forms X = R~^-T (J^T J) R~^-1 (close to the identity), its
// Cholesky factor X = L L^T, and R = L^T R~ -- all in FP64.  The Gram blocks
// are built from the input rows (FP32 inputs are widened exactly) with
// b_g = sqrt(m2_g) H(B_g) taken from the head/tail scan of B.
//
// Kernels: a tiled split-K Gram (each workgroup one 64 x 64 output tile over a
// chunk of rows; chunks summed afterwards in a fixed order), row-parallel
// triangular solves, a blocked right-looking Cholesky (one launch per block column), and a parallel
// triangular product.
#include "common.h"

#include <algorithm>
#include <cfloat>

namespace figaro {
namespace {

constexpr int kTile = 64;
constexpr int kRowsPerStage = 32;

// Group of row s of a table (groups given by start offsets and sizes); -1 if unmatched.
__device__ inline int group_of_row(const int32_t *off, const int32_t *size, int G, int64_t s)
{
    int lo = 0, hi = G;  // first group whose end > s
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((int64_t)off[mid] + size[mid] > s) hi = mid;
        else lo = mid + 1;
    }
    if (lo < G && off[lo] <= s) return lo;
    return -1;
}

// One output tile (ti, tj) of a Gram block over one chunk of rows:
// mode 0: C += w_r X_r^T X_r over rows of X (w_r = other[g(r)], the other table's group size)
// mode 1: C += X_r^T (sqrt(other[g]) hB[g]) over rows of X (the cross block, X = A)
template <typename Tin>
__device__ __forceinline__ void gram_tile(const GramJob &J, int ti, int tj, int chunk)
{
    // mode 0 is symmetric: only the tiles on or below the diagonal are formed
    if (J.mode == 0 && tj > ti) return;
    const Tin *__restrict__ X = (const Tin *)J.X;
    const int64_t ldx = J.ld;
    const int m = J.m, nx = J.nx, ny = J.ny, mode = J.mode;
    const int tid = threadIdx.x;
    const int G = (int)*J.Gp;
    const int64_t r0 = (int64_t)chunk * J.rows_per_chunk;
    int64_t r1 = min((int64_t)m, r0 + J.rows_per_chunk);
    if (mode == 2) r1 = min(r1, (int64_t)G);  // rows past the group count are empty
    __shared__ double xi[kRowsPerStage][kTile];
    __shared__ double yj[kRowsPerStage][kTile];
    __shared__ int grp[kRowsPerStage];
    // wave w accumulates the 16 x 16 subtiles (w, v), v = 0..3, of the 64 x 64 tile on the
    // FP64 matrix cores: D += A B with A = the i-columns of 4 staged rows transposed
    // (lane l supplies A[l % 16][l / 16]) and B = the j-columns (lane l supplies
    // B[l / 16][l % 16]); lane l holds D[l / 16 + 4 r][l % 16] in element r
    const int wv = tid >> 6, lane = tid & 63;
    typedef double d4 __attribute__((ext_vector_type(4)));
    d4 acc[4];
#pragma unroll
    for (int v = 0; v < 4; v++) acc[v] = d4{0.0, 0.0, 0.0, 0.0};
    const bool wlive = ti * kTile + wv * 16 < nx;
    const int vlive = min(4, ((mode == 0 ? nx : ny) - tj * kTile + 15) / 16);
    for (int64_t rb = r0; rb < r1; rb += kRowsPerStage) {
        if (tid < kRowsPerStage) {
            const int64_t s = rb + tid;
            // mode 2: rows are the groups themselves
            grp[tid] = s >= r1 ? -1
                       : mode == 2 ? (s < G ? (int)s : -1)
                       : J.cartesian ? (G > 0 ? 0 : -1)
                                     : group_of_row(J.off, J.size, G, s);
        }
        __syncthreads();
        // stage rows: i-columns of X, j-columns of X (weighted) or of the group's B sum.
        // Every load is issued unconditionally (row and column clamped into range) and
        // masked afterwards, so that a thread's loads are in flight together.
        constexpr int PER = kRowsPerStage * kTile / 256;
        double vi[PER], vj[PER];
#pragma unroll
        for (int u = 0; u < PER; u++) {
            const int e = tid + 256 * u, rr = e / kTile, c = e - rr * kTile;
            const int64_t s = min(rb + rr, r1 - 1);
            const int g = max(grp[rr], 0);
            const int ci = min(ti * kTile + c, nx - 1), cj = min(tj * kTile + c, (mode == 0 ? nx : ny) - 1);
            if (mode == 2) {
                // sum_g a_g b_g^T with a_g = sqrt(m1_g) H(A_g), b_g = sqrt(m2_g) H(B_g)
                vi[u] = sqrt((double)J.size[g]) * J.hA[(int64_t)g * nx + ci];
                vj[u] = sqrt((double)J.other[g]) * J.hB[(int64_t)g * ny + cj];
            } else if (mode == 0) {
                vi[u] = (double)X[s * ldx + ci];
                vj[u] = (double)J.other[g] * (double)X[s * ldx + cj];
            } else {
                vi[u] = (double)X[s * ldx + ci];
                vj[u] = sqrt((double)J.other[g]) * J.hB[(int64_t)g * ny + cj];
            }
        }
#pragma unroll
        for (int u = 0; u < PER; u++) {
            const int e = tid + 256 * u, rr = e / kTile, c = e - rr * kTile;
            const bool live = grp[rr] >= 0;
            xi[rr][c] = (live && ti * kTile + c < nx) ? vi[u] : 0.0;
            yj[rr][c] = (live && tj * kTile + c < (mode == 0 ? nx : ny)) ? vj[u] : 0.0;
        }
        __syncthreads();
        // subtiles wholly past the block's rows or columns (narrow tables) are skipped
        if (wlive) {
#pragma unroll
            for (int k0 = 0; k0 < kRowsPerStage; k0 += 4) {
                const double a = xi[k0 + lane / 16][wv * 16 + lane % 16];
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    if (v >= vlive) break;
                    const double b = yj[k0 + lane / 16][v * 16 + lane % 16];
                    acc[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[v], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    const int NY = mode == 0 ? nx : ny;
    double *out = J.partial + (int64_t)chunk * nx * NY;
#pragma unroll
    for (int v = 0; v < 4; v++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int i = ti * kTile + wv * 16 + lane / 16 + 4 * r, j = tj * kTile + v * 16 + lane % 16;
            if (i < nx && j < NY) out[(int64_t)i * NY + j] = acc[v][r];
        }
}

template <typename Tin>
__global__ __launch_bounds__(256) void k_gram_tile(GramJob J)
{
    gram_tile<Tin>(J, blockIdx.x, blockIdx.y, blockIdx.z);
}

// The tiles of a batch of Gram jobs: block b is tile (map[b].y, map[b].z) of chunk map[b].w
// of job map[b].x.
template <typename Tin>
__global__ __launch_bounds__(256) void k_gram_tile_batch(const GramJob *__restrict__ jobs, const int4 *__restrict__ map)
{
    const int4 e = map[blockIdx.x];
    const GramJob J = jobs[e.x];
    gram_tile<Tin>(J, e.y, e.z, e.w);
}

// Entry e of the job's Gram block at (row0, col0) of the N x N Gram (+ its transpose when
// mirror) = the sum of the job's chunk partials, in a fixed order.
__device__ __forceinline__ void gram_reduce(const GramJob &J, int64_t e)
{
    const int NY = J.mode == 0 ? J.nx : J.ny;
    const int64_t cnt = (int64_t)J.nx * NY;
    if (e >= cnt) return;
    const int i = (int)(e / NY), j = (int)(e - (int64_t)i * NY);
    // mode 0: an entry of a tile above the diagonal is read from its mirror image
    const int64_t src = (J.mode == 0 && j / kTile > i / kTile) ? (int64_t)j * NY + i : e;
    // eight interleaved partial sums (their loads in flight together), combined in a fixed order
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int c = 0;
    for (; c + 8 <= J.nch; c += 8)
#pragma unroll
        for (int u = 0; u < 8; u++) a[u] += J.partial[(int64_t)(c + u) * cnt + src];
    for (int u = 0; c < J.nch; c++, u++) a[u] += J.partial[(int64_t)c * cnt + src];
    const double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    J.gram[(int64_t)(J.row0 + i) * J.ldg + J.col0 + j] = s;
    if (J.mirror) J.gram[(int64_t)(J.col0 + j) * J.ldg + J.row0 + i] = s;
}

__global__ void k_gram_reduce(GramJob J)
{
    gram_reduce(J, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void k_gram_reduce_batch(const GramJob *__restrict__ jobs, const int2 *__restrict__ map)
{
    const int2 e = map[blockIdx.x];
    const GramJob J = jobs[e.x];
    gram_reduce(J, (int64_t)e.y * blockDim.x + threadIdx.x);
}

// Row i of Y = row i of G times Rt^-1 (Y Rt = G), Rt upper triangular; one workgroup per row.
// Column-oriented substitution: y = g; for k: y_k /= Rt_kk; y_{k+1:} -= y_k Rt_{k, k+1:}.
// transpose_in: read row i of G^T (column i of G) instead.
__global__ __launch_bounds__(256) void k_right_solve(const double *__restrict__ G, int ldg, const double *__restrict__ Rt,
                                                     int ldr, int n, double *__restrict__ Y, int ldy,
                                                     int transpose_in)
{
    extern __shared__ double y[];
    const int i = blockIdx.x;
    for (int k = threadIdx.x; k < n; k += blockDim.x)
        y[k] = transpose_in ? G[(int64_t)k * ldg + i] : G[(int64_t)i * ldg + k];
    __syncthreads();
    for (int k = 0; k < n; k++) {
        const double yk = y[k] / Rt[(int64_t)k * ldr + k];
        __syncthreads();
        for (int j = k + 1 + threadIdx.x; j < n; j += blockDim.x) y[j] -= yk * Rt[(int64_t)k * ldr + j];
        if (threadIdx.x == 0) y[k] = yk;
        __syncthreads();
    }
    for (int k = threadIdx.x; k < n; k += blockDim.x) Y[(int64_t)i * ldy + k] = y[k];
}

// Blocked right-looking Cholesky of (X + X^T) / 2 = L L^T, one launch per block column kb
// of kCb columns.  The launch reads block column kb of X (not written in the step) and
// updates the trailing lower blocks (i, j), kb < j <= i, each by one workgroup, which
// recomputes what it needs of block column kb: the diagonal factor L_kk (in LDS) and the
// panel blocks L_ik = X_ik L_kk^-T and L_jk.  Workgroup 0 stores L_kk, and workgroup
// (i, kb + 1) stores L_ik, into L (a separate buffer, so no block is read after it is
// overwritten).  Step 0 reads X symmetrised.  Padding past n acts as the identity.
// *failed <- 1 when a pivot is not a positive finite number (step 0 first sets it from
// its own pivots, so no clearing is needed), else it stays 0.
constexpr int kCb = 32;
__device__ inline double chol_load(const double *X, int ldx, int n, int r, int c, bool sym)
{
    if (r >= n || c >= n) return r == c ? 1.0 : 0.0;
    const double v = X[(int64_t)r * ldx + c];
    return sym ? 0.5 * (v + X[(int64_t)c * ldx + r]) : v;
}

__global__ __launch_bounds__(256) void k_chol_step(double *X, int ldx, int n, int kb, double *L, int ldl,
                                                   int32_t *failed)
{
    __shared__ double D[kCb][kCb + 1];
    __shared__ double P[2][kCb][kCb + 1];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const bool sym = kb == 0;
    const int nblk = (n + kCb - 1) / kCb;
    // block pair of this workgroup: 0 -> the diagonal factor only; else (i, j), kb < j <= i
    int bi = kb, bj = kb;
    if (blockIdx.x > 0) {
        int t = blockIdx.x - 1;
        bj = kb + 1;
        while (t >= nblk - bj) {
            t -= nblk - bj;
            bj++;
        }
        bi = bj + t;
    }
    const int k0 = kb * kCb, i0 = bi * kCb, j0 = bj * kCb;
    for (int e = tid; e < kCb * kCb; e += 256) {
        const int r = e / kCb, c = e - r * kCb;
        D[r][c] = c <= r ? chol_load(X, ldx, n, k0 + r, k0 + c, sym) : 0.0;
        if (blockIdx.x > 0) {
            P[0][r][c] = chol_load(X, ldx, n, i0 + r, k0 + c, sym);
            P[1][r][c] = chol_load(X, ldx, n, j0 + r, k0 + c, sym);
        }
    }
    __syncthreads();
    // diagonal factor by wave 0, lane r owning row r
    if (wv == 0) {
        int bad = 0;
        for (int c = 0; c < kCb; c++) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const double d = D[c][c];
            const bool ok = d > 0.0 && d <= DBL_MAX;
            const double p = ok ? sqrt(d) : 1.0;
            bad |= !ok;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (lane == c) D[c][c] = p;
            if (lane > c && lane < kCb) D[lane][c] /= p;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (lane > c && lane < kCb) {
                const double lr = D[lane][c];
                for (int cc = c + 1; cc <= lane; cc++) D[lane][cc] -= lr * D[cc][c];
            }
        }
        if (blockIdx.x == 0 && lane == 0 && (bad || kb == 0)) *failed = bad;
    }
    __syncthreads();
    if (blockIdx.x == 0) {
        for (int e = tid; e < kCb * kCb; e += 256) {
            const int r = e / kCb, c = e - r * kCb;
            if (k0 + r < n && k0 + c < n) L[(int64_t)(k0 + r) * ldl + k0 + c] = c <= r ? D[r][c] : 0.0;
        }
        return;
    }
    // panel blocks: row r of P[s] <- row r of X_(i or j),k times L_kk^-T (forward substitution)
    const bool same = bi == bj;
    if (tid < 2 * kCb && (tid < kCb || !same)) {
        const int s = tid / kCb, r = tid % kCb;
        double a[kCb];
#pragma unroll
        for (int c = 0; c < kCb; c++) a[c] = P[s][r][c];
#pragma unroll
        for (int c = 0; c < kCb; c++) {
            double v = a[c];
#pragma unroll
            for (int t = 0; t < c; t++) v = fma(-a[t], D[c][t], v);
            a[c] = v / D[c][c];
        }
#pragma unroll
        for (int c = 0; c < kCb; c++) P[s][r][c] = a[c];
    }
    __syncthreads();
    const int sj = same ? 0 : 1;
    if (bj == kb + 1) {
        for (int e = tid; e < kCb * kCb; e += 256) {
            const int r = e / kCb, c = e - r * kCb;
            if (i0 + r < n && k0 + c < n) L[(int64_t)(i0 + r) * ldl + k0 + c] = P[0][r][c];
        }
    }
    // X_ij -= L_ik L_jk^T (each thread four entries of one row); a diagonal block keeps its
    // upper part untouched (step 0 reads it as the transpose partner of the lower part)
    const int r = tid / 8, c0 = (tid % 8) * 4;
    double acc[4];
#pragma unroll
    for (int q = 0; q < 4; q++) acc[q] = chol_load(X, ldx, n, i0 + r, j0 + c0 + q, sym);
#pragma unroll 8
    for (int t = 0; t < kCb; t++) {
        const double lr = P[0][r][t];
#pragma unroll
        for (int q = 0; q < 4; q++) acc[q] = fma(-lr, P[sj][c0 + q][t], acc[q]);
    }
    if (i0 + r < n) {
#pragma unroll
        for (int q = 0; q < 4; q++)
            if (j0 + c0 + q < n && (!same || c0 + q <= r)) X[(int64_t)(i0 + r) * ldx + j0 + c0 + q] = acc[q];
    }
}

// R = L^T Rt (both triangular): R_ij = sum_{k=i..j} L_ki Rt_kj, zeros below the diagonal.
// When the Cholesky step failed, R = Rt (the sweep is skipped).
__global__ void k_lt_times_r(const double *__restrict__ L, int ldl, const double *__restrict__ Rt, int ldt, int n,
                             const int32_t *failed, double *__restrict__ R, int64_t ldr)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * n) return;
    const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
    double s = 0.0;
    if (*failed) {
        s = Rt[(int64_t)i * ldt + j];
    } else if (j >= i) {
        for (int k = i; k <= j; k++) s = fma(L[(int64_t)k * ldl + i], Rt[(int64_t)k * ldt + j], s);
    }
    R[(int64_t)i * ldr + j] = s;
}

// The whole N x N part in one workgroup for N <= 128, with the triangles in LDS:
//   1. T = R~^-1 (upper): R~ staged in LDS, then thread j forms column j by back
//      substitution (t_j = 1 / R~_jj, t_k = -(sum_{l=k+1..j} R~_kl t_l) / R~_kk);
//   2. Y = Gram T (through global scratch, every thread a set of entries);
//   3. X = T^T Y, lower triangle only (X is symmetric in exact arithmetic);
//   4. right-looking Cholesky X = L L^T in LDS;
//   5. R = L^T R~.
// A zero or non-finite pivot (R~ singular to working precision) skips the sweep: R = R~.
constexpr int kSmallMax = 128;
constexpr int kSmallThreads = 1024;
__device__ inline int lpk(int i, int j) { return i * (i + 1) / 2 + j; }       // lower packed, j <= i
__device__ inline int upk(int n, int i, int j) { return i * n - i * (i - 1) / 2 + (j - i); }  // upper, j >= i

__device__ __forceinline__ void refine_small(const double *__restrict__ gram, const double *__restrict__ Rt, int ldt,
                                             int n, double *__restrict__ Y, int32_t *failed, double *__restrict__ R,
                                             int64_t ldr)
{
    __shared__ double Tu[kSmallMax * (kSmallMax + 1) / 2];  // R~, then R~^-1 (upper, packed)
    __shared__ double Xl[kSmallMax * (kSmallMax + 1) / 2];  // R~ staged, then X and L (lower, packed)
    __shared__ double piv;
    __shared__ int bad;
    const int tid = threadIdx.x, nt = blockDim.x;
    // R~ (upper) staged into Xl's space, read as R~_kl = Xl[upk(n, k, l)]
    for (int e = tid; e < n * n; e += nt) {
        const int i = e / n, j = e - i * n;
        if (j >= i) Xl[upk(n, i, j)] = Rt[(int64_t)i * ldt + j];
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    if (tid < n) {
        const int j = tid;
        Tu[upk(n, j, j)] = 1.0 / Xl[upk(n, j, j)];
        for (int k = j - 1; k >= 0; k--) {
            double a0 = 0.0, a1 = 0.0;
            int l = k + 1;
            for (; l + 1 <= j; l += 2) {
                a0 = fma(Xl[upk(n, k, l)], Tu[upk(n, l, j)], a0);
                a1 = fma(Xl[upk(n, k, l + 1)], Tu[upk(n, l + 1, j)], a1);
            }
            if (l <= j) a0 = fma(Xl[upk(n, k, l)], Tu[upk(n, l, j)], a0);
            Tu[upk(n, k, j)] = -(a0 + a1) / Xl[upk(n, k, k)];
        }
    }
    __syncthreads();
    // Y = Gram T: Y_ij = sum_{k <= j} G_ik T_kj
    for (int e = tid; e < n * n; e += nt) {
        const int i = e / n, j = e - i * n;
        const double *g = gram + (int64_t)i * n;
        double a0 = 0.0, a1 = 0.0;
        int k = 0;
        for (; k + 1 <= j; k += 2) {
            a0 = fma(g[k], Tu[upk(n, k, j)], a0);
            a1 = fma(g[k + 1], Tu[upk(n, k + 1, j)], a1);
        }
        if (k <= j) a0 = fma(g[k], Tu[upk(n, k, j)], a0);
        Y[(int64_t)i * n + j] = a0 + a1;
    }
    __syncthreads();
    // X = T^T Y, lower: X_ij = sum_{k <= i} T_ki Y_kj (j <= i)
    for (int e = tid; e < n * n; e += nt) {
        const int i = e / n, j = e - i * n;
        if (j > i) continue;
        double a0 = 0.0, a1 = 0.0;
        int k = 0;
        for (; k + 1 <= i; k += 2) {
            a0 = fma(Tu[upk(n, k, i)], Y[(int64_t)k * n + j], a0);
            a1 = fma(Tu[upk(n, k + 1, i)], Y[(int64_t)(k + 1) * n + j], a1);
        }
        if (k <= i) a0 = fma(Tu[upk(n, k, i)], Y[(int64_t)k * n + j], a0);
        Xl[lpk(i, j)] = a0 + a1;
    }
    __syncthreads();
    for (int k = 0; k < n; k++) {
        if (tid == 0) {
            const double d = Xl[lpk(k, k)];
            const bool ok = d > 0.0 && d <= DBL_MAX;
            piv = ok ? sqrt(d) : 1.0;
            if (!ok) bad = 1;
            Xl[lpk(k, k)] = piv;
        }
        __syncthreads();
        const double p = piv;
        for (int i = k + 1 + tid; i < n; i += nt) Xl[lpk(i, k)] /= p;
        __syncthreads();
        const int rem = n - k - 1;
        for (int e = tid; e < rem * rem; e += nt) {
            const int i = k + 1 + e / rem, j = k + 1 + e % rem;
            if (j <= i) Xl[lpk(i, j)] -= Xl[lpk(i, k)] * Xl[lpk(j, k)];
        }
        __syncthreads();
    }
    const bool fail = bad != 0;
    if (tid == 0) *failed = bad;
    for (int e = tid; e < n * n; e += nt) {
        const int i = e / n, j = e - i * n;
        double v = 0.0;
        if (fail) {
            v = j >= i ? Rt[(int64_t)i * ldt + j] : 0.0;
        } else if (j >= i) {
            for (int k = i; k <= j; k++) v = fma(Xl[lpk(k, i)], Rt[(int64_t)k * ldt + j], v);
        }
        R[(int64_t)i * ldr + j] = v;
    }
}

__global__ __launch_bounds__(kSmallThreads) void k_refine_small(const double *__restrict__ gram,
                                                               const double *__restrict__ Rt, int ldt, int n,
                                                               double *__restrict__ Y, int32_t *failed,
                                                               double *__restrict__ R, int64_t ldr)
{
    refine_small(gram, Rt, ldt, n, Y, failed, R, ldr);
}

// One workgroup per instance of a batch.
__global__ __launch_bounds__(kSmallThreads) void k_refine_small_batch(const RefineSmall *__restrict__ tab)
{
    const RefineSmall j = tab[blockIdx.x];
    refine_small(j.gram, j.Rt, j.ldt, j.n, j.Y, j.failed, j.R, j.ldr);
}

// Row chunks of a Gram block: about `blocks` workgroups per block (1024 for a single
// problem; a batch, whose jobs fill the GPU together, asks for fewer), at least 256 rows each.
constexpr int64_t kGramBlocks = 1024, kGramMinRows = 256;
int64_t gram_chunks(int64_t m, int64_t tiles, int64_t blocks)
{
    const int64_t c = std::min<int64_t>((m + kGramMinRows - 1) / kGramMinRows, (blocks + tiles - 1) / tiles);
    return std::max<int64_t>(c, 1);
}

int64_t gram_need(int64_t nx, int64_t ny)
{
    const int64_t tiles = ((nx + kTile - 1) / kTile) * ((ny + kTile - 1) / kTile);
    return (kGramBlocks + tiles - 1) / tiles * nx * ny;
}

}  // namespace

int gram_jobs(const void *A, int in_f64, int64_t lda, int64_t m1, int n1, const void *B, int64_t ldb, int64_t m2,
              int n2, Groups g, int cartesian, const double *hA, const double *hB, int64_t gcap, double *partial,
              double *gram, GramJob *jobs, int64_t blocks)
{
    const int N = n1 + n2;
    const int64_t p0 = gram_need(n1, n1), p1 = gram_need(n2, n2);
    struct Spec {
        const void *X;
        int64_t ld, m;
        int nx, ny, mode;
        const int32_t *off, *size, *other;
        int row0, col0, mirror;
        double *part;
    };
    const Spec spec[3] = {
        {A, lda, m1, n1, n1, 0, g.offA, g.m1, g.m2, 0, 0, 0, partial},
        {B, ldb, m2, n2, n2, 0, g.offB, g.m2, g.m1, n1, n1, 0, partial + p0},
        hA ? Spec{nullptr, 0, gcap, n1, n2, 2, g.offA, g.m1, g.m2, 0, n1, 1, partial + p0 + p1}
           : Spec{A, lda, m1, n1, n2, 1, g.offA, g.m1, g.m2, 0, n1, 1, partial + p0 + p1},
    };
    for (int k = 0; k < 3; k++) {
        const Spec &sp = spec[k];
        GramJob &J = jobs[k];
        J.X = sp.X;
        J.ld = sp.ld;
        J.m = (int32_t)sp.m;
        J.nx = sp.nx;
        J.ny = sp.ny;
        J.mode = sp.mode;
        J.in_f64 = in_f64;
        J.off = sp.off;
        J.size = sp.size;
        J.other = sp.other;
        J.Gp = g.counts + CNT_G;
        J.cartesian = cartesian;
        J.hA = hA;
        J.hB = hB;
        J.gx = (sp.nx + kTile - 1) / kTile;
        J.gy = (sp.ny + kTile - 1) / kTile;
        J.nch = (int32_t)gram_chunks(sp.m, (int64_t)J.gx * J.gy, std::min(blocks, kGramBlocks));
        J.rows_per_chunk = (sp.m + J.nch - 1) / J.nch;
        J.partial = sp.part;
        J.gram = gram;
        J.ldg = N;
        J.row0 = sp.row0;
        J.col0 = sp.col0;
        J.mirror = sp.mirror;
    }
    return 3;
}

hipError_t launch_gram_batch(int in_f64, const GramJob *jobs, const int4 *tile_map, int64_t ntiles,
                             const int2 *red_map, int64_t nred, hipStream_t s)
{
    if (ntiles == 0) return hipSuccess;
    if (in_f64) k_gram_tile_batch<double><<<(unsigned)ntiles, 256, 0, s>>>(jobs, tile_map);
    else k_gram_tile_batch<float><<<(unsigned)ntiles, 256, 0, s>>>(jobs, tile_map);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_gram_reduce_batch<<<(unsigned)nred, 256, 0, s>>>(jobs, red_map);
    return hipGetLastError();
}

namespace {

}  // namespace

int64_t refine_partial_elems(int64_t n1, int64_t n2)
{
    // the partial sums of the three Gram blocks, side by side
    return gram_need(n1, n1) + gram_need(n2, n2) + gram_need(n1, n2);
}

hipError_t launch_refine_small_batch(const RefineSmall *tab, int count, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    k_refine_small_batch<<<(unsigned)count, kSmallThreads, 0, s>>>(tab);
    return hipGetLastError();
}

hipError_t launch_refine(const void *A, int in_f64, int64_t lda, int64_t m1, int n1, const void *B,
                         int64_t ldb, int64_t m2, int n2, Groups g, int cartesian, const double *hA,
                         const double *hB, int64_t gcap,
                         const double *Rt, int ldt, double *gram, double *Y, double *partial,
                         int64_t partial_cap, int32_t *failed, double *R, int64_t ldr, hipStream_t s, int part)
{
    const int N = n1 + n2;
    if (partial_cap < refine_partial_elems(n1, n2)) return hipErrorInvalidValue;
    GramJob jobs[3];
    gram_jobs(A, in_f64, lda, m1, n1, B, ldb, m2, n2, g, cartesian, hA, hB, gcap, partial, gram, jobs, kGramBlocks);
    for (const GramJob &J : jobs) {
        if (part == 1) break;
        dim3 grid(J.gx, J.gy, (unsigned)J.nch);
        if (in_f64) k_gram_tile<double><<<grid, 256, 0, s>>>(J);
        else k_gram_tile<float><<<grid, 256, 0, s>>>(J);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int64_t out_elems = (int64_t)J.nx * (J.mode == 0 ? J.nx : J.ny);
        k_gram_reduce<<<(unsigned)((out_elems + 255) / 256), 256, 0, s>>>(J);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (part == 0) return hipSuccess;
    if (N <= kSmallMax) {
        k_refine_small<<<1, kSmallThreads, 0, s>>>(gram, Rt, ldt, N, Y, failed, R, ldr);
        return hipGetLastError();
    }
    const size_t shm = sizeof(double) * N;
    // Y = Gram Rt^-1 ; then X^T = Y^T Rt^-1 (X symmetric), written over gram
    k_right_solve<<<N, 256, shm, s>>>(gram, N, Rt, ldt, N, Y, N, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_right_solve<<<N, 256, shm, s>>>(Y, N, Rt, ldt, N, gram, N, 1);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // L (lower) into Y's space: Y is not read again
    const int nblk = (N + kCb - 1) / kCb;
    for (int kb = 0; kb < nblk; kb++) {
        const int rem = nblk - kb - 1;
        k_chol_step<<<(unsigned)(1 + rem * (rem + 1) / 2), 256, 0, s>>>(gram, N, N, kb, Y, N, failed);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int64_t nn = (int64_t)N * N;
    k_lt_times_r<<<(unsigned)((nn + 255) / 256), 256, 0, s>>>(Y, N, Rt, ldt, N, failed, R, ldr);
    return hipGetLastError();
}

}  // namespace figaro
