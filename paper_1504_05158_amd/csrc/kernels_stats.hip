// Population statistics of goals (Sec. 4.2): percentile ranks and PMF counts,
// per swarm and over the whole population, computed on demand or recorded at
// every iteration into a ring of records (k_history).
//
// k_select: the value of a given rank in a segment of int64 values, by an
// MSD radix select over the 64-bit key (sign bit flipped, which orders signed
// values as unsigned): 8 passes, each counting the next byte of the keys that
// share the prefix fixed so far (LDS histogram), then descending into the byte
// that holds the rank.  One workgroup per (segment, rank).
//
// k_hist: per segment, the counts of values in bins ((g - lo) * bins) / (hi - lo)
// for lo <= g < hi, accumulated in LDS.  One workgroup per segment.
#include "kernels.hpp"

namespace qap {

// The value at 1-based position r (1 <= r <= e - b) of values[b, e) in
// ascending order; one workgroup, result returned to every thread.
__device__ long long select_rank(const long long* __restrict__ values, int b, int e, long long r)
{
    __shared__ unsigned cnt[256];
    __shared__ unsigned long long s_prefix;
    __shared__ long long s_rank;
    unsigned long long prefix = 0, mask = 0;
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 56 - 8 * pass;
        for (int i = threadIdx.x; i < 256; i += blockDim.x) cnt[i] = 0;
        __syncthreads();
        for (int i = b + (int)threadIdx.x; i < e; i += blockDim.x) {
            const unsigned long long key = (unsigned long long)values[i] ^ (1ull << 63);
            if ((key & mask) == prefix) atomicAdd(&cnt[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            long long rr = r;
            int digit = 0;
            while (digit < 255 && rr > (long long)cnt[digit]) {
                rr -= cnt[digit];
                ++digit;
            }
            s_prefix = prefix | ((unsigned long long)digit << shift);
            s_rank = rr;
        }
        __syncthreads();
        prefix = s_prefix;
        r = s_rank;
        mask |= 255ull << shift;
        __syncthreads();
    }
    return (long long)(prefix ^ (1ull << 63));
}

__global__ __launch_bounds__(256) void k_select(const long long* __restrict__ values, const int* __restrict__ seg_off,
                                                const long long* __restrict__ ranks, int nr,
                                                long long* __restrict__ out)
{
    const int seg = (int)blockIdx.x / nr;
    const long long v = select_rank(values, seg_off[seg], seg_off[seg + 1], ranks[blockIdx.x]);
    if (threadIdx.x == 0) out[blockIdx.x] = v;
}

// Counts of values[b, e) in bins ((g - lo) * bins) / (hi - lo) for lo <= g < hi
// into out [bins]; one workgroup, hist: its LDS counters [bins].
__device__ void hist_segment(const long long* __restrict__ values, int b, int e, int bins, long long lo, long long hi,
                             unsigned* hist, unsigned long long* __restrict__ out)
{
    for (int i = threadIdx.x; i < bins; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const long long width = hi - lo;
    for (int i = b + (int)threadIdx.x; i < e; i += blockDim.x) {
        const long long g = values[i];
        if (g >= lo && g < hi) atomicAdd(&hist[(int)(((g - lo) * bins) / width)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < bins; i += blockDim.x) out[i] = hist[i];
}

__global__ __launch_bounds__(256) void k_hist(const long long* __restrict__ values, const int* __restrict__ seg_off,
                                              int bins, long long lo, long long hi,
                                              unsigned long long* __restrict__ out)
{
    extern __shared__ unsigned hist[];
    const int seg = (int)blockIdx.x;
    hist_segment(values, seg_off[seg], seg_off[seg + 1], bins, lo, hi, hist, out + (size_t)seg * bins);
}

// ------------------------------------------------------------------ history
// One record of the per-iteration statistics of an instance (m swarms of S
// particles, P = m S): segments 0 .. m - 1 are the swarms, segment m the
// population.  The record goes to slot (t - 1) % capacity of the ring, t the
// instance's iteration counter after the step (read on the device): ring_t
// [capacity], ring_q [capacity][m + 1][nq] (ranks of each segment in
// ranks [(m + 1) nq]), ring_h [capacity][m + 1][bins].  Workgroups 0 ..
// (m + 1) nq - 1 select, the next m + 1 count.
__global__ __launch_bounds__(256) void k_history(const long long* __restrict__ goals, const int* __restrict__ iter,
                                                 int m, int S, int nq, const long long* __restrict__ ranks, int bins,
                                                 long long lo, long long hi, int capacity, int* __restrict__ ring_t,
                                                 long long* __restrict__ ring_q,
                                                 unsigned long long* __restrict__ ring_h)
{
    extern __shared__ unsigned hist[];
    const int t = *iter;
    const int slot = (t - 1) % capacity;
    const int nsel = (m + 1) * nq;
    const int blk = (int)blockIdx.x;
    if (blk < nsel) {
        const int seg = blk / nq;
        const int b = seg < m ? seg * S : 0, e = seg < m ? (seg + 1) * S : m * S;
        const long long v = select_rank(goals, b, e, ranks[blk]);
        if (threadIdx.x == 0) ring_q[(size_t)slot * nsel + blk] = v;
    } else {
        const int seg = blk - nsel;
        const int b = seg < m ? seg * S : 0, e = seg < m ? (seg + 1) * S : m * S;
        hist_segment(goals, b, e, bins, lo, hi, hist, ring_h + ((size_t)slot * (m + 1) + seg) * bins);
    }
    if (blk == 0 && threadIdx.x == 0) ring_t[slot] = t;
}

hipError_t launch_history(const long long* goals, const int* iter, int m, int S, int nq, const long long* ranks,
                          int bins, long long lo, long long hi, int capacity, int* ring_t, long long* ring_q,
                          unsigned long long* ring_h, hipStream_t st)
{
    const int blocks = (m + 1) * nq + (bins > 0 ? m + 1 : 0);
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_history, dim3((unsigned)blocks), dim3(256), sizeof(unsigned) * (size_t)(bins > 0 ? bins : 1),
                       st, goals, iter, m, S, nq, ranks, bins, lo, hi, capacity, ring_t, ring_q, ring_h);
    return hipGetLastError();
}

// Segment offsets and ranks of a statistics request, written on the device:
// seg_off [m + 3] = (0, S, .., m S) for the m swarms, then (0, P) for the
// population; ranks [(m + 1) nq] = max(1, ceil(q_j N / 10^6)) with N = S for
// the swarms and P for the population.
__global__ void k_stats_setup(int* __restrict__ seg_off, long long* __restrict__ ranks, int m, int S, int P, int nq,
                              StatsRanks q)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i <= m) seg_off[i] = i * S;
    if (i == m + 1) seg_off[i] = 0;
    if (i == m + 2) seg_off[i] = P;
    if (i < (m + 1) * nq) {
        const int g = i / nq, j = i % nq;
        const long long N = g < m ? S : P;
        const long long r = ((long long)q.ppm[j] * N + 999999) / 1000000;
        ranks[i] = r > 1 ? r : 1;
    }
}

hipError_t launch_stats_setup(int* seg_off, long long* ranks, int m, int S, int P, int nq, const StatsRanks& q,
                              hipStream_t st)
{
    const long long items = (long long)(m + 3) > (long long)(m + 1) * nq ? (long long)(m + 3) : (long long)(m + 1) * nq;
    hipLaunchKernelGGL(k_stats_setup, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, st, seg_off, ranks, m, S, P,
                       nq, q);
    return hipGetLastError();
}

hipError_t launch_select(const long long* values, const int* seg_off, int nseg, const long long* ranks, int nr,
                         long long* out, hipStream_t st)
{
    if (nseg <= 0 || nr <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_select, dim3((unsigned)(nseg * nr)), dim3(256), 0, st, values, seg_off, ranks, nr, out);
    return hipGetLastError();
}

hipError_t launch_hist(const long long* values, const int* seg_off, int nseg, int bins, long long lo, long long hi,
                       unsigned long long* out, hipStream_t st)
{
    if (nseg <= 0 || bins <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_hist, dim3((unsigned)nseg), dim3(256), sizeof(unsigned) * (size_t)bins, st, values, seg_off,
                       bins, lo, hi, out);
    return hipGetLastError();
}

}  // namespace qap
