// Stable sort of a table's rows by its int32 join key, on the device.
//
// The method takes its relations sorted by the join attribute (Experiments
// section); this lifts that precondition.  Keys are mapped to unsigned order
// (sign bit flipped) and sorted together with their row indices by a least-
// significant-digit radix sort of 4-bit digits (8 passes).  Each pass:
//   1. count: every block of 2048 keys counts its 16 digit values;
//   2. scan: one workgroup turns the counts (digit-major, then block) into the
//      exclusive start of every (digit, block) pair;
//   3. scatter: every block ranks its keys within each digit in input order
//      (per-thread counts, then a block scan per digit) and writes key and index
//      to start + rank.
// Equal keys keep their input order in every pass, so the whole sort is stable.
// The rows are then gathered in the sorted order.
#include "common.h"

#include <algorithm>

namespace figaro {
namespace {

constexpr int kSortThreads = 256;
constexpr int kSortPer = 8;  // keys per thread
constexpr int kSortBlock = kSortThreads * kSortPer;
constexpr int kDigits = 16;
constexpr int kPasses = 8;

__device__ inline uint32_t ukey(int32_t k) { return (uint32_t)k ^ 0x80000000u; }

// Pass p reads the flipped keys from `kin` (pass 0: the table's keys) and counts digit
// (key >> shift) & 15 of block b into counts[digit * nblocks + b].
__global__ __launch_bounds__(kSortThreads) void k_sort_count(const uint32_t *__restrict__ kin,
                                                             const int32_t *__restrict__ keys0, int64_t n, int shift,
                                                             int32_t *__restrict__ counts, int nblocks)
{
    __shared__ int32_t h[kDigits];
    if (threadIdx.x < kDigits) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortBlock + (int64_t)threadIdx.x * kSortPer;
    for (int u = 0; u < kSortPer; u++) {
        const int64_t i = base + u;
        if (i < n) {
            const uint32_t k = keys0 ? ukey(keys0[i]) : kin[i];
            atomicAdd(&h[(k >> shift) & (kDigits - 1)], 1);
        }
    }
    __syncthreads();
    if (threadIdx.x < kDigits) counts[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of counts[0 .. total) in place, one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_sort_scan(int32_t *counts, int64_t total)
{
    __shared__ int32_t s[1024];
    int32_t carry = 0;
    for (int64_t b0 = 0; b0 < total; b0 += 1024) {
        const int64_t i = b0 + threadIdx.x;
        const int32_t v = i < total ? counts[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int32_t a = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += a;
            __syncthreads();
        }
        if (i < total) counts[i] = carry + s[threadIdx.x] - v;
        carry += s[1023];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(const uint32_t *__restrict__ kin,
                                                               const int32_t *__restrict__ iin,
                                                               const int32_t *__restrict__ keys0, int64_t n, int shift,
                                                               const int32_t *__restrict__ starts, int nblocks,
                                                               uint32_t *__restrict__ kout, int32_t *__restrict__ iout)
{
    __shared__ int32_t t[kDigits][kSortThreads];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kSortBlock + (int64_t)tid * kSortPer;
    uint32_t k[kSortPer];
    int32_t idx[kSortPer];
    int32_t c[kDigits];
#pragma unroll
    for (int d = 0; d < kDigits; d++) c[d] = 0;
#pragma unroll
    for (int u = 0; u < kSortPer; u++) {
        const int64_t i = base + u;
        const bool in = i < n;
        k[u] = in ? (keys0 ? ukey(keys0[i]) : kin[i]) : 0u;
        idx[u] = in ? (keys0 ? (int32_t)i : iin[i]) : -1;
        if (in) {
            const int d = (k[u] >> shift) & (kDigits - 1);
#pragma unroll
            for (int e = 0; e < kDigits; e++) c[e] += (e == d);
        }
    }
#pragma unroll
    for (int d = 0; d < kDigits; d++) t[d][tid] = c[d];
    __syncthreads();
    // inclusive scan along the threads, every digit at once (Hillis-Steele)
    for (int off = 1; off < kSortThreads; off <<= 1) {
        int32_t a[kDigits];
#pragma unroll
        for (int d = 0; d < kDigits; d++) a[d] = tid >= off ? t[d][tid - off] : 0;
        __syncthreads();
#pragma unroll
        for (int d = 0; d < kDigits; d++) t[d][tid] += a[d];
        __syncthreads();
    }
    int32_t pos[kDigits];
#pragma unroll
    for (int d = 0; d < kDigits; d++) pos[d] = starts[(int64_t)d * nblocks + blockIdx.x] + t[d][tid] - c[d];
#pragma unroll
    for (int u = 0; u < kSortPer; u++) {
        if (idx[u] < 0) continue;
        const int d = (k[u] >> shift) & (kDigits - 1);
        int32_t p = 0;
#pragma unroll
        for (int e = 0; e < kDigits; e++)
            if (e == d) p = pos[e]++;
        kout[p] = k[u];
        iout[p] = idx[u];
    }
}

// out row r = in row perm[r]; keys_out[r] = the signed key.
template <typename T>
__global__ void k_gather_rows(const T *__restrict__ in, int64_t ld_in, int64_t cols, const int32_t *__restrict__ perm,
                              const uint32_t *__restrict__ ksorted, int64_t n, T *__restrict__ out, int64_t ld_out,
                              int32_t *__restrict__ keys_out)
{
    const int64_t r = blockIdx.x;
    if (r >= n) return;
    const int64_t src = perm[r];
    for (int64_t c = threadIdx.x; c < cols; c += blockDim.x) out[r * ld_out + c] = in[src * ld_in + c];
    if (threadIdx.x == 0 && keys_out) keys_out[r] = (int32_t)(ksorted[r] ^ 0x80000000u);
}

}  // namespace

int64_t sort_workspace_bytes(int64_t n)
{
    const int64_t nb = (n + kSortBlock - 1) / kSortBlock;
    // two key buffers, two index buffers, the (digit, block) counts; 256-byte aligned pieces
    auto al = [](int64_t b) { return (b + 255) / 256 * 256; };
    return 2 * al(4 * std::max<int64_t>(n, 1)) + 2 * al(4 * std::max<int64_t>(n, 1)) +
           al(4 * (int64_t)kDigits * std::max<int64_t>(nb, 1));
}

hipError_t launch_sort_table(const void *X, int elem_bytes, int64_t ld, int64_t n, int64_t cols, const int32_t *keys,
                             void *out, int64_t ld_out, int32_t *keys_out, void *ws, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    if (n > INT32_MAX) return hipErrorInvalidValue;
    const int nb = (int)((n + kSortBlock - 1) / kSortBlock);
    auto al = [](int64_t b) { return (b + 255) / 256 * 256; };
    char *p = (char *)ws;
    uint32_t *ka = (uint32_t *)p;
    p += al(4 * n);
    uint32_t *kb = (uint32_t *)p;
    p += al(4 * n);
    int32_t *ia = (int32_t *)p;
    p += al(4 * n);
    int32_t *ib = (int32_t *)p;
    p += al(4 * n);
    int32_t *counts = (int32_t *)p;
    const uint32_t *kin = nullptr;
    const int32_t *iin = nullptr;
    uint32_t *kout = ka;
    int32_t *iout = ia;
    for (int pass = 0; pass < kPasses; pass++) {
        const int shift = 4 * pass;
        const int32_t *k0 = pass == 0 ? keys : nullptr;
        k_sort_count<<<nb, kSortThreads, 0, s>>>(kin, k0, n, shift, counts, nb);
        k_sort_scan<<<1, 1024, 0, s>>>(counts, (int64_t)kDigits * nb);
        k_sort_scatter<<<nb, kSortThreads, 0, s>>>(kin, iin, k0, n, shift, counts, nb, kout, iout);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        kin = kout;
        iin = iout;
        kout = kout == ka ? kb : ka;
        iout = iout == ia ? ib : ia;
    }
    // after an even number of passes the result is back in the first pair of buffers
    if (elem_bytes == 8)
        k_gather_rows<double><<<(unsigned)n, 64, 0, s>>>((const double *)X, ld, cols, iin, kin, n, (double *)out,
                                                        ld_out, keys_out);
    else
        k_gather_rows<float><<<(unsigned)n, 64, 0, s>>>((const float *)X, ld, cols, iin, kin, n, (float *)out, ld_out,
                                                       keys_out);
    return hipGetLastError();
}

}  // namespace figaro
