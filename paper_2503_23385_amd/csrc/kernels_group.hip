// Key grouping on the device (integer work, bit-exact).
//
// The paper's inputs are sorted by the join attribute (Experiments
// section); the natural join then decomposes into one Cartesian product per
// key present in both tables (Section 1, Claim 1 applied per key group).
// This file turns two non-decreasing int32 key columns into the group table
// {key, offA, m1_g, offB, m2_g, r1_g, r2_g} in ascending key order, with
//   r1_g = sum_{h<g} m1_h,  r2_g = sum_{h<g} (m2_h - 1),
//   counts = {G, R1 = sum m1_g, R2 = sum (m2_g - 1), join_rows = sum m1_g m2_g}.
//
// Three block-scan rounds: (1) run starts of each key column, (2) runs of A
// matched against runs of B by binary search, (3) exclusive sums of the
// matched group sizes.  Each round is count -> single-workgroup scan -> apply.
#include "common.h"

namespace figaro {
namespace {

constexpr int EPT = kGroupBlock / kGroupThreads;  // elements per thread (8)

__global__ void k_init(int32_t *status, int64_t *counts, int32_t *ticket, int32_t *flags,
                       int64_t nflags)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        *status = kStatusOk;
        for (int c = 0; c < CNT_SLOTS; c++) counts[c] = 0;
        if (ticket) *ticket = 0;
    }
    for (int64_t j = i; j < nflags; j += (int64_t)gridDim.x * blockDim.x) flags[j] = 0;
}

// The one-group table of a Cartesian product, its counts and status (one thread).
__device__ inline void cartesian_table(int32_t *status, Groups g, int64_t m1, int64_t m2)
{
    *status = kStatusOk;
    for (int c = 0; c < CNT_SLOTS; c++) g.counts[c] = 0;
    const bool nonempty = m1 > 0 && m2 > 0;
    g.counts[CNT_G] = nonempty ? 1 : 0;
    g.counts[CNT_R1] = nonempty ? m1 : 0;
    g.counts[CNT_R2] = nonempty ? m2 - 1 : 0;
    g.counts[CNT_JOIN] = nonempty ? m1 * m2 : 0;
    g.counts[CNT_TA] = nonempty ? m1 - 1 : 0;
    g.key[0] = 0;
    g.offA[0] = 0;
    g.m1[0] = (int32_t)m1;
    g.offB[0] = 0;
    g.m2[0] = (int32_t)m2;
    g.r1[0] = 0;
    g.r2[0] = 0;
}

// The whole grouping of a Cartesian product (one group) with the initialisation of
// k_init in the same launch: node counters zeroed by every thread, the status, counts
// and the one-group table written by thread 0.
__global__ void k_cartesian(int32_t *status, int32_t *flags, int64_t nflags, Groups g, int64_t m1, int64_t m2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t j = i; j < nflags; j += (int64_t)gridDim.x * blockDim.x) flags[j] = 0;
    if (i == 0) cartesian_table(status, g, m1, m2);
}

// A batch of Cartesian instances, one workgroup each: its counters zeroed, its table set.
__global__ void k_cartesian_batch(const CartInit *__restrict__ tab)
{
    const CartInit c = tab[blockIdx.x];
    for (int64_t j = threadIdx.x; j < c.nflags; j += blockDim.x) c.flags[j] = 0;
    if (threadIdx.x == 0) cartesian_table(c.status, c.g, c.m1, c.m2);
}

// Workgroup exclusive scan of one int per thread; returns the prefix and sets *total.
template <typename T>
__device__ T block_exclusive_scan(T v, T *lds, T *total)
{
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = 1; off < (int)blockDim.x; off <<= 1) {
        T add = (t >= off) ? lds[t - off] : T(0);
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    T incl = lds[t];
    *total = lds[blockDim.x - 1];
    __syncthreads();
    return incl - v;
}

// Pass 1a: run starts per block, and sortedness.  Blocks [0, nbA) scan A, the rest B.
__global__ __launch_bounds__(kGroupThreads) void k_run_count(const int32_t *kA, int64_t m1,
                                                             const int32_t *kB, int64_t m2,
                                                             int nbA, int32_t *blkA, int32_t *blkB,
                                                             int32_t *status)
{
    const bool isA = (int)blockIdx.x < nbA;
    const int b = isA ? blockIdx.x : blockIdx.x - nbA;
    const int32_t *k = isA ? kA : kB;
    const int64_t m = isA ? m1 : m2;
    const int64_t i0 = (int64_t)b * kGroupBlock + (int64_t)threadIdx.x * EPT;
    int cnt = 0;
    bool bad = false;
    for (int e = 0; e < EPT; e++) {
        const int64_t i = i0 + e;
        if (i < m) {
            const int32_t cur = k[i];
            if (i == 0) cnt++;
            else {
                const int32_t prev = k[i - 1];
                cnt += (cur != prev);
                bad |= (cur < prev);
            }
        }
    }
    if (bad) atomicExch(status, kStatusUnsorted);
    __shared__ int lds[kGroupThreads];
    int tot;
    block_exclusive_scan<int>(cnt, lds, &tot);
    if (threadIdx.x == 0) (isA ? blkA : blkB)[b] = tot;
}

// Single workgroup (1024 threads): exclusive scan in place of arr[0..n); total to *total.
// blockIdx.x selects one of two independent arrays.
template <typename T>
__global__ __launch_bounds__(1024) void k_scan_small(T *arr0, int n0, int64_t *total0, T *arr1,
                                                     int n1, int64_t *total1, int32_t *sent0,
                                                     int64_t sentval0, int32_t *sent1,
                                                     int64_t sentval1)
{
    T *arr = blockIdx.x == 0 ? arr0 : arr1;
    const int n = blockIdx.x == 0 ? n0 : n1;
    int64_t *total = blockIdx.x == 0 ? total0 : total1;
    int32_t *sent = blockIdx.x == 0 ? sent0 : sent1;
    const int64_t sentval = blockIdx.x == 0 ? sentval0 : sentval1;
    if (arr == nullptr) return;
    __shared__ T lds[1024];
    T carry = 0;
    for (int base = 0; base < n; base += 1024) {
        const int i = base + threadIdx.x;
        T v = i < n ? arr[i] : T(0);
        T tot;
        T ex = block_exclusive_scan<T>(v, lds, &tot);
        if (i < n) arr[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        if (total) *total = (int64_t)carry;
        // run-start arrays get a sentinel run_start[U] = m
        if (sent) sent[(int64_t)carry] = (int32_t)sentval;
    }
}

// Pass 1b: scatter the first row index of every run.
__global__ __launch_bounds__(kGroupThreads) void k_run_scatter(const int32_t *kA, int64_t m1,
                                                               const int32_t *kB, int64_t m2,
                                                               int nbA, const int32_t *blkA,
                                                               const int32_t *blkB, int32_t *runA,
                                                               int32_t *runB)
{
    const bool isA = (int)blockIdx.x < nbA;
    const int b = isA ? blockIdx.x : blockIdx.x - nbA;
    const int32_t *k = isA ? kA : kB;
    const int64_t m = isA ? m1 : m2;
    int32_t *run = isA ? runA : runB;
    const int32_t base = (isA ? blkA : blkB)[b];
    const int64_t i0 = (int64_t)b * kGroupBlock + (int64_t)threadIdx.x * EPT;
    int cnt = 0;
    for (int e = 0; e < EPT; e++) {
        const int64_t i = i0 + e;
        if (i < m) cnt += (i == 0) || (k[i] != k[i - 1]);
    }
    __shared__ int lds[kGroupThreads];
    int tot;
    int pos = base + block_exclusive_scan<int>(cnt, lds, &tot);
    for (int e = 0; e < EPT; e++) {
        const int64_t i = i0 + e;
        if (i < m && ((i == 0) || (k[i] != k[i - 1]))) run[pos++] = (int32_t)i;
    }
}

// Pass 2a: match each run of A against the runs of B (binary search on run keys).
// With unsorted keys (status set by pass 1a) no run matches: a key may then recur in
// several runs, and the sizes the later rounds derive from matches would no longer be
// bounded by the group table's and the regions' capacities.  The join is taken as empty.
__global__ __launch_bounds__(kGroupThreads) void k_match(const int32_t *kA, const int32_t *runA,
                                                         const int64_t *UAp, const int32_t *kB,
                                                         const int32_t *runB, const int64_t *UBp,
                                                         const int32_t *status, int32_t *matchA,
                                                         int32_t *blkM)
{
    const int64_t UA = *UAp, UB = *status == kStatusOk ? *UBp : 0;
    const int64_t u0 = (int64_t)blockIdx.x * kGroupBlock + (int64_t)threadIdx.x * EPT;
    int cnt = 0;
    for (int e = 0; e < EPT; e++) {
        const int64_t u = u0 + e;
        if (u >= UA) break;
        const int32_t key = kA[runA[u]];
        int64_t lo = 0, hi = UB;  // first run of B with key >= key
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (kB[runB[mid]] < key) lo = mid + 1;
            else hi = mid;
        }
        const int32_t v = (lo < UB && kB[runB[lo]] == key) ? (int32_t)lo : -1;
        matchA[u] = v;
        cnt += v >= 0;
    }
    __shared__ int lds[kGroupThreads];
    int tot;
    block_exclusive_scan<int>(cnt, lds, &tot);
    if (threadIdx.x == 0) blkM[blockIdx.x] = tot;
}

// Pass 2b: emit groups; per-block sums of m1_g, m2_g - 1 and m1_g * m2_g.
__global__ __launch_bounds__(kGroupThreads) void k_group_emit(
    const int32_t *kA, const int32_t *runA, const int64_t *UAp, const int32_t *runB,
    const int32_t *matchA, const int32_t *blkM, Groups g, int64_t *blkS, int nb)
{
    const int64_t UA = *UAp;
    const int64_t u0 = (int64_t)blockIdx.x * kGroupBlock + (int64_t)threadIdx.x * EPT;
    int cnt = 0;
    for (int e = 0; e < EPT; e++) {
        const int64_t u = u0 + e;
        if (u < UA) cnt += matchA[u] >= 0;
    }
    __shared__ int lds[kGroupThreads];
    int tot;
    int gi = blkM[blockIdx.x] + block_exclusive_scan<int>(cnt, lds, &tot);
    int64_t s1 = 0, s2 = 0, sj = 0;
    for (int e = 0; e < EPT; e++) {
        const int64_t u = u0 + e;
        if (u >= UA) break;
        const int32_t v = matchA[u];
        if (v < 0) continue;
        const int32_t a0 = runA[u], a1 = runA[u + 1];
        const int32_t b0 = runB[v], b1 = runB[v + 1];
        g.key[gi] = kA[a0];
        g.offA[gi] = a0;
        g.m1[gi] = a1 - a0;
        g.offB[gi] = b0;
        g.m2[gi] = b1 - b0;
        s1 += a1 - a0;
        s2 += (b1 - b0) - 1;
        sj += (int64_t)(a1 - a0) * (int64_t)(b1 - b0);
        gi++;
    }
    __shared__ int64_t l64[kGroupThreads];
    int64_t t1, t2, tj;
    block_exclusive_scan<int64_t>(s1, l64, &t1);
    block_exclusive_scan<int64_t>(s2, l64, &t2);
    block_exclusive_scan<int64_t>(sj, l64, &tj);
    if (threadIdx.x == 0) {
        blkS[blockIdx.x] = t1;
        blkS[nb + blockIdx.x] = t2;
        blkS[2 * nb + blockIdx.x] = tj;
    }
}

// Single workgroup: exclusive scans of the three per-block sums; totals to counts.
__global__ __launch_bounds__(1024) void k_scan_sums(int64_t *blkS, int nb, int64_t *counts)
{
    __shared__ int64_t lds[1024];
    for (int a = 0; a < 3; a++) {
        int64_t *arr = blkS + (int64_t)a * nb;
        int64_t carry = 0;
        for (int base = 0; base < nb; base += 1024) {
            const int i = base + threadIdx.x;
            int64_t v = i < nb ? arr[i] : 0;
            int64_t tot;
            int64_t ex = block_exclusive_scan<int64_t>(v, lds, &tot);
            if (i < nb) arr[i] = carry + ex;
            carry += tot;
        }
        if (threadIdx.x == 0) counts[a == 0 ? CNT_R1 : (a == 1 ? CNT_R2 : CNT_JOIN)] = carry;
    }
}

// Pass 3: r1_g, r2_g from the block offsets and a block-local scan.
__global__ __launch_bounds__(kGroupThreads) void k_group_offsets(const int64_t *UAp,
                                                                 const int32_t *matchA,
                                                                 const int32_t *blkM,
                                                                 const int64_t *blkS, int nb,
                                                                 Groups g)
{
    const int64_t UA = *UAp;
    const int64_t u0 = (int64_t)blockIdx.x * kGroupBlock + (int64_t)threadIdx.x * EPT;
    int cnt = 0;
    for (int e = 0; e < EPT; e++) {
        const int64_t u = u0 + e;
        if (u < UA) cnt += matchA[u] >= 0;
    }
    __shared__ int lds[kGroupThreads];
    int tot;
    const int g0 = blkM[blockIdx.x] + block_exclusive_scan<int>(cnt, lds, &tot);
    int64_t s1 = 0, s2 = 0;
    for (int c = 0; c < cnt; c++) {
        s1 += g.m1[g0 + c];
        s2 += g.m2[g0 + c] - 1;
    }
    __shared__ int64_t l64[kGroupThreads];
    int64_t t1, t2;
    int64_t e1 = block_exclusive_scan<int64_t>(s1, l64, &t1) + blkS[blockIdx.x];
    int64_t e2 = block_exclusive_scan<int64_t>(s2, l64, &t2) + blkS[nb + blockIdx.x];
    for (int c = 0; c < cnt; c++) {
        const int gi = g0 + c;
        g.r1[gi] = (int32_t)e1;
        g.r2[gi] = (int32_t)e2;
        e1 += g.m1[gi];
        e2 += g.m2[gi] - 1;
    }
}

__global__ void k_set_G(const int64_t *Gtot, int64_t *counts)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        counts[CNT_G] = *Gtot;
        counts[CNT_TA] = counts[CNT_R1] - *Gtot;
    }
}

}  // namespace

hipError_t launch_group_init(int32_t *status, int64_t *counts, int32_t *ticket, int32_t *flags,
                             int64_t nflags, hipStream_t s)
{
    int64_t blocks = (nflags + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    k_init<<<(unsigned)blocks, 256, 0, s>>>(status, counts, ticket, flags, nflags);
    return hipGetLastError();
}

hipError_t launch_group_cartesian(int32_t *status, int32_t *flags, int64_t nflags, Groups g, int64_t m1,
                                  int64_t m2, hipStream_t s)
{
    int64_t blocks = (nflags + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    k_cartesian<<<(unsigned)blocks, 256, 0, s>>>(status, flags, nflags, g, m1, m2);
    return hipGetLastError();
}

hipError_t launch_group_cartesian_batch(const CartInit *tab, int count, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    k_cartesian_batch<<<(unsigned)count, 256, 0, s>>>(tab);
    return hipGetLastError();
}

hipError_t launch_group_keys(const int32_t *kA, int64_t m1, const int32_t *kB, int64_t m2,
                             Groups g, int32_t *blkA, int32_t *blkB, int32_t *runA, int32_t *runB,
                             int32_t *matchA, int32_t *blkM, int64_t *blkS, int32_t *status,
                             hipStream_t s)
{
    const int nbA = (int)((m1 + kGroupBlock - 1) / kGroupBlock);
    const int nbB = (int)((m2 + kGroupBlock - 1) / kGroupBlock);
    if (nbA + nbB == 0) return hipSuccess;
    int64_t *counts = g.counts;
    k_run_count<<<nbA + nbB, kGroupThreads, 0, s>>>(kA, m1, kB, m2, nbA, blkA, blkB, status);
    k_scan_small<int32_t><<<2, 1024, 0, s>>>(blkA, nbA, counts + CNT_UA, blkB, nbB,
                                             counts + CNT_UB, runA, m1, runB, m2);
    k_run_scatter<<<nbA + nbB, kGroupThreads, 0, s>>>(kA, m1, kB, m2, nbA, blkA, blkB, runA, runB);
    if (nbA == 0 || nbB == 0) return hipGetLastError();
    k_match<<<nbA, kGroupThreads, 0, s>>>(kA, runA, counts + CNT_UA, kB, runB, counts + CNT_UB,
                                          status, matchA, blkM);
    // G lands in counts[CNT_G] via the scan total (CNT_TMP used as a temporary).
    k_scan_small<int32_t><<<1, 1024, 0, s>>>(blkM, nbA, counts + CNT_TMP, nullptr, 0, nullptr, nullptr, 0,
                                             nullptr, 0);
    k_group_emit<<<nbA, kGroupThreads, 0, s>>>(kA, runA, counts + CNT_UA, runB, matchA, blkM, g,
                                               blkS, nbA);
    k_scan_sums<<<1, 1024, 0, s>>>(blkS, nbA, counts);
    k_group_offsets<<<nbA, kGroupThreads, 0, s>>>(counts + CNT_UA, matchA, blkM, blkS, nbA, g);
    k_set_G<<<1, 64, 0, s>>>(counts + CNT_TMP, counts);
    return hipGetLastError();
}

}  // namespace figaro
