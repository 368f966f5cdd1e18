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
// triangular solves, a one-workgroup right-looking Cholesky, and a parallel
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

// mode 0: C += w_r X_r^T X_r over rows of X (w_r = other[g(r)], the other table's group size)
// mode 1: C += X_r^T (sqrt(other[g]) hB[g]) over rows of X (the cross block, X = A)
template <typename Tin, int MODE>
__global__ __launch_bounds__(256) void k_gram_tile(const Tin *__restrict__ X, int64_t ldx, int m, int nx,
                                                   const int32_t *off, const int32_t *size,
                                                   const int32_t *other, const int64_t *Gp,
                                                   int cartesian, const double *__restrict__ hB, int ny,
                                                   int64_t rows_per_chunk, double *__restrict__ partial)
{
    const int ti = blockIdx.x, tj = blockIdx.y, chunk = blockIdx.z;
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;  // 16 x 16 threads, 4 x 4 outputs each
    const int G = (int)*Gp;
    const int64_t r0 = (int64_t)chunk * rows_per_chunk;
    const int64_t r1 = min((int64_t)m, r0 + rows_per_chunk);
    __shared__ double xi[kRowsPerStage][kTile];
    __shared__ double yj[kRowsPerStage][kTile];
    __shared__ int grp[kRowsPerStage];
    double acc[4][4] = {};
    for (int64_t rb = r0; rb < r1; rb += kRowsPerStage) {
        if (tid < kRowsPerStage) {
            const int64_t s = rb + tid;
            grp[tid] = s >= r1 ? -1 : cartesian ? (G > 0 ? 0 : -1) : group_of_row(off, size, G, s);
        }
        __syncthreads();
        // stage rows: i-columns of X, j-columns of X (weighted) or of the group's B sum
#pragma unroll 4
        for (int e = tid; e < kRowsPerStage * kTile; e += 256) {
            const int rr = e / kTile, c = e - rr * kTile;
            const int64_t s = rb + rr;
            double vi = 0.0, vj = 0.0;
            {
                const int g = grp[rr];
                if (g >= 0) {
                    const int ci = ti * kTile + c, cj = tj * kTile + c;
                    if (ci < nx) vi = (double)X[s * ldx + ci];
                    if (MODE == 0) {
                        if (cj < nx) vj = (double)other[g] * (double)X[s * ldx + cj];
                    } else {
                        if (cj < ny) vj = sqrt((double)other[g]) * hB[(int64_t)g * ny + cj];
                    }
                }
            }
            xi[rr][c] = vi;
            yj[rr][c] = vj;
        }
        __syncthreads();
#pragma unroll 4
        for (int rr = 0; rr < kRowsPerStage; rr++) {
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                a[u] = xi[rr][ty * 4 + u];
                b[u] = yj[rr][tx * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; u++)
#pragma unroll
                for (int v = 0; v < 4; v++) acc[u][v] = fma(a[u], b[v], acc[u][v]);
        }
        __syncthreads();
    }
    const int NY = MODE == 0 ? nx : ny;
    double *out = partial + (int64_t)chunk * nx * NY;
#pragma unroll
    for (int u = 0; u < 4; u++)
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int i = ti * kTile + ty * 4 + u, j = tj * kTile + tx * 4 + v;
            if (i < nx && j < NY) out[(int64_t)i * NY + j] = acc[u][v];
        }
}

// Gram(N x N) block at (row0, col0) (+ its transpose when `mirror`) = sum of chunks, fixed order.
__global__ void k_gram_reduce(const double *__restrict__ partial, int nchunks, int rows, int cols,
                              double *__restrict__ gram, int ldg, int row0, int col0, int mirror)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * cols) return;
    double s = 0.0;
    for (int c = 0; c < nchunks; c++) s += partial[(int64_t)c * rows * cols + e];
    const int i = (int)(e / cols), j = (int)(e - (int64_t)i * cols);
    gram[(int64_t)(row0 + i) * ldg + col0 + j] = s;
    if (mirror) gram[(int64_t)(col0 + j) * ldg + row0 + i] = s;
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

// In place: X <- lower Cholesky factor of (X + X^T) / 2 (one workgroup, right-looking).
// *failed <- 1 when a pivot is not a positive finite number (R~ singular to working
// precision, e.g. a rank-deficient join), else 0.
__global__ __launch_bounds__(1024) void k_cholesky(double *X, int ldx, int n, int32_t *failed)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int e = tid; e < n * n; e += nt) {
        const int i = e / n, j = e - i * n;
        if (i > j) {
            const double s = 0.5 * (X[(int64_t)i * ldx + j] + X[(int64_t)j * ldx + i]);
            X[(int64_t)i * ldx + j] = s;
        }
    }
    __syncthreads();
    __shared__ double piv;
    __shared__ int bad;
    if (tid == 0) bad = 0;
    for (int k = 0; k < n; k++) {
        if (tid == 0) {
            const double d = X[(int64_t)k * ldx + k];
            const bool ok = d > 0.0 && d <= DBL_MAX;
            piv = ok ? sqrt(d) : 1.0;
            if (!ok) bad = 1;
            X[(int64_t)k * ldx + k] = piv;
        }
        __syncthreads();
        const double p = piv;
        for (int i = k + 1 + tid; i < n; i += nt) X[(int64_t)i * ldx + k] /= p;
        __syncthreads();
        const int rem = n - k - 1;
        for (int e = tid; e < rem * rem; e += nt) {
            const int i = k + 1 + e / rem, j = k + 1 + e % rem;
            if (j <= i) X[(int64_t)i * ldx + j] -= X[(int64_t)i * ldx + k] * X[(int64_t)j * ldx + k];
        }
        __syncthreads();
    }
    if (tid == 0) *failed = bad;
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

// The whole N x N part in one workgroup for N <= 128: R~ and the lower triangle of X
// live in LDS (packed), Y = Gram R~^-1 goes through global scratch.
//   1. row i (one thread each): y = g_i R~^-1 by forward substitution;
//   2. column j (one thread each, in place over Y): x = R~^-T y_:,j; keep k >= j;
//   3. right-looking Cholesky of X in LDS;
//   4. R = L^T R~.
constexpr int kSmallMax = 128;
__device__ inline int lpk(int i, int j) { return i * (i + 1) / 2 + j; }       // lower packed, j <= i
__device__ inline int upk(int n, int i, int j) { return i * n - i * (i - 1) / 2 + (j - i); }  // upper, j >= i

__global__ __launch_bounds__(1024) void k_refine_small(const double *__restrict__ gram, const double *__restrict__ Rt,
                                                       int ldt, int n, double *__restrict__ Y,
                                                       int32_t *failed, double *__restrict__ R, int64_t ldr)
{
    __shared__ double Ru[kSmallMax * (kSmallMax + 1) / 2];
    __shared__ double Xl[kSmallMax * (kSmallMax + 1) / 2];
    __shared__ double piv;
    __shared__ int bad;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int e = tid; e < n * n; e += nt) {
        const int i = e / n, j = e - i * n;
        if (j >= i) Ru[upk(n, i, j)] = Rt[(int64_t)i * ldt + j];
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    if (tid < n) {  // row tid of Y: y_k = (g_k - sum_{l<k} y_l R_lk) / R_kk
        const int i = tid;
        for (int k = 0; k < n; k++) {
            double acc = gram[(int64_t)i * n + k];
            for (int l = 0; l < k; l++) acc = fma(-Y[(int64_t)i * n + l], Ru[upk(n, l, k)], acc);
            Y[(int64_t)i * n + k] = acc / Ru[upk(n, k, k)];
        }
    }
    __syncthreads();
    if (tid < n) {  // column tid of X, in place over Y: x_k = (y_kj - sum_{l<k} R_lk x_l) / R_kk
        const int j = tid;
        for (int k = 0; k < n; k++) {
            double acc = Y[(int64_t)k * n + j];
            for (int l = 0; l < k; l++) acc = fma(-Ru[upk(n, l, k)], Y[(int64_t)l * n + j], acc);
            const double xk = acc / Ru[upk(n, k, k)];
            Y[(int64_t)k * n + j] = xk;
            if (k >= j) Xl[lpk(k, j)] = xk;
        }
    }
    __syncthreads();
    // X is symmetric in exact arithmetic; its lower triangle (from the column solves) is used.
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
        for (int e = tid; e < rem * (rem + 1) / 2; e += nt) {
            // e -> (i, j) with k < j <= i < n
            int i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
            while ((i + 1) * (i + 2) / 2 <= e) i++;
            while (i * (i + 1) / 2 > e) i--;
            const int j = e - i * (i + 1) / 2;
            const int ii = k + 1 + i, jj = k + 1 + j;
            Xl[lpk(ii, jj)] -= Xl[lpk(ii, k)] * Xl[lpk(jj, k)];
        }
        __syncthreads();
    }
    const bool fail = bad != 0;
    if (tid == 0) *failed = bad;
    for (int e = tid; e < n * n; e += nt) {
        const int i = e / n, j = e - i * n;
        double s = 0.0;
        if (fail) {
            s = j >= i ? Ru[upk(n, i, j)] : 0.0;
        } else if (j >= i) {
            for (int k = i; k <= j; k++) s = fma(Xl[lpk(k, i)], Ru[upk(n, k, j)], s);
        }
        R[(int64_t)i * ldr + j] = s;
    }
}

template <typename Tin>
hipError_t gram_blocks(const void *A, int64_t lda, int64_t m1, int n1, const void *B, int64_t ldb,
                       int64_t m2, int n2, Groups g, int cartesian, const double *hB, double *partial,
                       int64_t partial_cap, double *gram, hipStream_t s)
{
    const int N = n1 + n2;
    // Row chunks: about 2048 workgroups in all, at least 256 rows each, partials within the cap.
    auto chunks_for = [&](int64_t m, int64_t tiles, int64_t out_elems) {
        int64_t c = std::min<int64_t>((m + 255) / 256, (2048 + tiles - 1) / tiles);
        c = std::min<int64_t>(c, partial_cap / out_elems);
        return std::max<int64_t>(c, 1);
    };
    struct Job { const Tin *X; int64_t ld, m; int nx, ny, mode; const int32_t *off, *size, *other; int row0, col0, mirror; };
    Job jobs[3] = {
        {(const Tin *)A, lda, m1, n1, n1, 0, g.offA, g.m1, g.m2, 0, 0, 0},
        {(const Tin *)B, ldb, m2, n2, n2, 0, g.offB, g.m2, g.m1, n1, n1, 0},
        {(const Tin *)A, lda, m1, n1, n2, 1, g.offA, g.m1, g.m2, 0, n1, 1},
    };
    for (const Job &jb : jobs) {
        const int gx = (jb.nx + kTile - 1) / kTile, gy = (jb.ny + kTile - 1) / kTile;
        const int64_t out_elems = (int64_t)jb.nx * jb.ny;
        const int64_t nch = chunks_for(jb.m, (int64_t)gx * gy, out_elems);
        const int64_t per = (jb.m + nch - 1) / nch;
        dim3 grid(gx, gy, (unsigned)nch);
        if (jb.mode == 0)
            k_gram_tile<Tin, 0><<<grid, 256, 0, s>>>(jb.X, jb.ld, (int)jb.m, jb.nx, jb.off, jb.size,
                                                     jb.other, g.counts + CNT_G, cartesian, hB, jb.ny, per, partial);
        else
            k_gram_tile<Tin, 1><<<grid, 256, 0, s>>>(jb.X, jb.ld, (int)jb.m, jb.nx, jb.off, jb.size,
                                                     jb.other, g.counts + CNT_G, cartesian, hB, jb.ny, per, partial);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        k_gram_reduce<<<(unsigned)((out_elems + 255) / 256), 256, 0, s>>>(partial, (int)nch, jb.nx, jb.ny, gram,
                                                                         N, jb.row0, jb.col0, jb.mirror);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

int64_t refine_partial_elems(int64_t n1, int64_t n2)
{
    // the most any Gram block asks for: ceil(2048 / tiles) chunks of nx * ny partial sums
    auto need = [](int64_t nx, int64_t ny) {
        const int64_t tiles = ((nx + kTile - 1) / kTile) * ((ny + kTile - 1) / kTile);
        return (2048 + tiles - 1) / tiles * nx * ny;
    };
    return std::max(need(n1, n1), std::max(need(n2, n2), need(n1, n2)));
}

hipError_t launch_refine(const void *A, int in_f64, int64_t lda, int64_t m1, int n1, const void *B,
                         int64_t ldb, int64_t m2, int n2, Groups g, int cartesian, const double *hB,
                         const double *Rt, int ldt, double *gram, double *Y, double *partial,
                         int64_t partial_cap, int32_t *failed, double *R, int64_t ldr, hipStream_t s)
{
    const int N = n1 + n2;
    hipError_t e = in_f64 ? gram_blocks<double>(A, lda, m1, n1, B, ldb, m2, n2, g, cartesian, hB, partial,
                                                partial_cap, gram, s)
                          : gram_blocks<float>(A, lda, m1, n1, B, ldb, m2, n2, g, cartesian, hB, partial,
                                               partial_cap, gram, s);
    if (e != hipSuccess) return e;
    if (N <= kSmallMax) {
        k_refine_small<<<1, 1024, 0, s>>>(gram, Rt, ldt, N, Y, failed, R, ldr);
        return hipGetLastError();
    }
    const size_t shm = sizeof(double) * N;
    // Y = Gram Rt^-1 ; then X^T = Y^T Rt^-1 (X symmetric), written over gram
    k_right_solve<<<N, 256, shm, s>>>(gram, N, Rt, ldt, N, Y, N, 0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_right_solve<<<N, 256, shm, s>>>(Y, N, Rt, ldt, N, gram, N, 1);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_cholesky<<<1, 1024, 0, s>>>(gram, N, N, failed);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nn = (int64_t)N * N;
    k_lt_times_r<<<(unsigned)((nn + 255) / 256), 256, 0, s>>>(gram, N, Rt, ldt, N, failed, R, ldr);
    return hipGetLastError();
}

}  // namespace figaro
