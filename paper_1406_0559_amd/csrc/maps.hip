// HIP kernels for the statistics and storage of finished maps on gfx950:
// normalisation to magnification and map statistics (eq. 4), count histograms, binned magnification probability distributions and
// probability sums (Vernardos & Fluke 2014, Section 3.2.1 and Section 4), the
// mean and spread of MPDs over lens realisations, and the indexed-map codec
// (Appendix B). All are single passes over the int32 count map, bound by HBM
// bandwidth; every decision that floating point takes is an FP64 comparison
// made the same way as in a plain sequential evaluation.
#include <climits>

#include "maps.h"

namespace rl {
namespace {

constexpr int kInFlight = 4;   // 16-byte loads in flight per thread

// Calls f(v) for every count of c[0 .. n) once, over the whole grid: 16-byte
// vector loads for the aligned body, kInFlight of them in flight per thread
// (the grids are a few waves per SIMD, so the loads of one thread must overlap),
// and scalar loads for the few counts before and after it. The order of the
// calls is unspecified; the callers only count and compare.
template <typename F>
__device__ __forceinline__ void grid_counts(const int32_t* __restrict__ c, int64_t n, F&& f) {
    const uintptr_t addr = reinterpret_cast<uintptr_t>(c);
    int64_t head = (int64_t)(((16u - (unsigned)(addr & 15u)) & 15u) >> 2);
    if (head > n) head = n;
    const int64_t nv = (n - head) >> 2;
    const int64_t tail0 = head + nv * 4;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    const int4* __restrict__ v = reinterpret_cast<const int4*>(c + head);
    int64_t k = tid;
    for (; k + (kInFlight - 1) * nth < nv; k += kInFlight * nth) {
        int4 q[kInFlight];
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) q[u] = v[k + u * nth];
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) {
            f(q[u].x);
            f(q[u].y);
            f(q[u].z);
            f(q[u].w);
        }
    }
    for (; k < nv; k += nth) {
        const int4 q = v[k];
        f(q.x);
        f(q.y);
        f(q.z);
        f(q.w);
    }
    if (tid < head) f(c[tid]);
    if (tid < n - tail0) f(c[tail0 + tid]);
}

// ----------------------------------------------------------------------------
// normalisation and map statistics (eq. 4)
// ----------------------------------------------------------------------------

__global__ void normalise_kernel(const int32_t* __restrict__ counts, int64_t n, double n_avg,
                                 float* __restrict__ mu) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
        mu[k] = (float)((double)counts[k] / n_avg);
}

__global__ void __launch_bounds__(256) count_stats_kernel(const int32_t* __restrict__ counts,
                                                          int64_t n,
                                                          const unsigned long long* __restrict__ escaped,
                                                          unsigned long long* __restrict__ out) {
    __shared__ unsigned long long ssum[4];
    __shared__ unsigned long long sneg[4];
    __shared__ int smax[4];
    unsigned long long s = 0, neg = 0;
    int mx = 0;
    grid_counts(counts, n, [&](int v) {
        if (v < 0) neg += 1;
        else s += (unsigned long long)(unsigned)v;
        mx = v > mx ? v : mx;
    });
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        s += __shfl_xor(s, o);
        neg += __shfl_xor(neg, o);
        const int t = __shfl_xor(mx, o);
        mx = t > mx ? t : mx;
    }
    const int w = threadIdx.x / kLanes;
    if ((threadIdx.x % kLanes) == 0) { ssum[w] = s; sneg[w] = neg; smax[w] = mx; }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long bs = 0, bn = 0;
        int bm = 0;
        for (int i = 0; i < (int)(blockDim.x / kLanes); ++i) {
            bs += ssum[i];
            bn += sneg[i];
            bm = smax[i] > bm ? smax[i] : bm;
        }
        unsigned long long* o = out + (int64_t)blockIdx.x * kRecWords;
        o[0] = bs;
        o[1] = (unsigned long long)bm;
        o[2] = bn;
        if (escaped && blockIdx.x == 0) out[(int64_t)kRedBlocks * kRecWords] = *escaped;
    }
}


// ----------------------------------------------------------------------------
// magnification probability distributions (Section 3.2.1 and Section 4)
// ----------------------------------------------------------------------------

constexpr int kHistLds = 16384;  // LDS words for the per-workgroup histogram copies
constexpr int kMaxReps = 32;     // copies of a histogram in LDS
// Histogram workgroups: 1024 threads (16 waves, 64 loads of 16 bytes in flight
// per SIMD) with 64 KiB of LDS copies, one or two per CU: few workgroups keep
// the flush (one device atomic per entry per workgroup) small.
constexpr int kHistThreads = 1024;
constexpr int kHistBlocks = 256;

// Copies of an LDS histogram of `slots` entries that fit in kHistLds words
// (a power of two, at most kMaxReps). Lane l adds into copy l % reps, stored
// interleaved (entry e of copy r at e * reps + r): lanes that hit the same
// entry then hit different words in different banks, so the LDS atomics of
// the few entries most pixels share do not serialise.
int hist_reps(int64_t slots, int64_t words = kHistLds) {
    int r = kMaxReps;
    while (r > 1 && slots * r > words) r >>= 1;
    return r;
}

// Frequency of each count value; values >= n_values - 1 share the last entry.
// Values below kHistLds / reps (where almost every pixel lies) go to LDS
// copies first, the rest straight to global atomics.
__global__ void __launch_bounds__(kHistThreads) count_hist_kernel(const int32_t* __restrict__ counts,
                                                         int64_t n, int64_t n_values, int reps,
                                                         unsigned long long* __restrict__ hist) {
    extern __shared__ __align__(16) unsigned int sh[];
    const int cap = kHistLds / reps;
    const int nl = (int)(n_values < cap ? n_values : cap);
    for (int e = threadIdx.x; e < nl * reps; e += blockDim.x) sh[e] = 0;
    __syncthreads();
    const int64_t last = n_values - 1;
    const int r = threadIdx.x & (reps - 1);
    grid_counts(counts, n, [&](int cv) {
        const int64_t c = cv < 0 ? 0 : cv;
        const int64_t v = c < last ? c : last;
        if (v < nl) atomicAdd(&sh[v * reps + r], 1u);
        else atomicAdd(&hist[v], 1ull);
    });
    __syncthreads();
    for (int e = threadIdx.x; e < nl; e += blockDim.x) {
        unsigned long long t = 0;
        for (int q = 0; q < reps; ++q) t += sh[e * reps + q];
        if (t) atomicAdd(&hist[e], t);
    }
}

// Bin of a count: the number of thresholds <= N (thresholds ascending), so
// bin 0 is the underflow and bin nthr the overflow.
__device__ __forceinline__ int mpd_bin(const double* __restrict__ st, int nthr, double c) {
    int lo = 0, hi = nthr;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (st[mid] <= c) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Binned MPD. Thresholds, the value table (the bin of every count below
// kMpdLut: counts are integers, so each value's decision is taken once per
// workgroup instead of once per pixel) and `reps` interleaved copies of the
// bins (as in count_hist_kernel) live in LDS; counts outside [0, kMpdLut) are
// searched directly. The thresholds come from the kernel argument when there
// are at most kMpdArgThr of them, else from thr.
__global__ void __launch_bounds__(kHistThreads) mpd_kernel(const int32_t* __restrict__ counts, int64_t n,
                                                  MpdThresholds targ, const double* __restrict__ thr,
                                                  int nthr, int reps,
                                                  unsigned long long* __restrict__ bins) {
    extern __shared__ __align__(16) char smem[];
    double* st = reinterpret_cast<double*>(smem);
    unsigned int* sb = reinterpret_cast<unsigned int*>(st + nthr);
    uint16_t* sl = reinterpret_cast<uint16_t*>(sb + (nthr + 1) * reps);
    const bool in_arg = nthr <= kMpdArgThr;
    for (int e = threadIdx.x; e < nthr; e += blockDim.x) st[e] = in_arg ? targ.t[e] : thr[e];
    for (int e = threadIdx.x; e < (nthr + 1) * reps; e += blockDim.x) sb[e] = 0;
    __syncthreads();
    for (int e = threadIdx.x; e < kMpdLut; e += blockDim.x) sl[e] = (uint16_t)mpd_bin(st, nthr, (double)e);
    __syncthreads();
    const int r = threadIdx.x & (reps - 1);
    grid_counts(counts, n, [&](int cv) {
        const int b = (unsigned)cv < (unsigned)kMpdLut ? (int)sl[cv] : mpd_bin(st, nthr, (double)cv);
        atomicAdd(&sb[b * reps + r], 1u);
    });
    __syncthreads();
    for (int e = threadIdx.x; e <= nthr; e += blockDim.x) {
        unsigned long long t = 0;
        for (int q = 0; q < reps; ++q) t += sb[e * reps + q];
        if (t) atomicAdd(&bins[e], t);
    }
}

// Calls f(v) for every value of x[0 .. n) once, over the whole grid, with
// 16-byte loads (two values) for the aligned body, kInFlight in flight per
// thread, and scalar loads for a leading value and the last one.
template <typename F>
__device__ __forceinline__ void grid_values(const double* __restrict__ x, int64_t n, F&& f) {
    const uintptr_t addr = reinterpret_cast<uintptr_t>(x);
    int64_t head = (addr & 15u) ? 1 : 0;
    if (head > n) head = n;
    const int64_t nv = (n - head) >> 1;
    const int64_t tail0 = head + nv * 2;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    const double2* __restrict__ v = reinterpret_cast<const double2*>(x + head);
    int64_t k = tid;
    for (; k + (kInFlight - 1) * nth < nv; k += kInFlight * nth) {
        double2 q[kInFlight];
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) q[u] = v[k + u * nth];
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) {
            f(q[u].x);
            f(q[u].y);
        }
    }
    for (; k < nv; k += nth) {
        const double2 q = v[k];
        f(q.x);
        f(q.y);
    }
    if (tid < head) f(x[tid]);
    if (tid < n - tail0) f(x[tail0 + tid]);
}

// Binned MPD of a map of real magnifications (a finite-source map): the bin
// of a value is the number of thresholds at or below it (NaN: none), found by
// a binary search in LDS; bins counted in `reps` interleaved LDS copies as in
// mpd_kernel. Thresholds from the kernel argument (at most kMpdArgThr) or thr.
// The bin is first guessed from an FP32 logarithm, g = floor((log10 mu - c0)
// * inv_step) + 1 clamped to [0, nthr] (c0 = log10 mu_ref + log_lo, inv_step =
// nbins / (log_hi - log_lo)), and kept only if the FP64 thresholds on either
// side confirm it, T_(g-1) <= mu < T_g; otherwise the binary search decides.
// The result is the threshold rule's in every case: the guess only saves the
// search. Values that are not > 0 (zero, negative, NaN) take bin 0 at once.
__device__ __forceinline__ int mpd_value_bin(const double* __restrict__ st, int nthr, double x, float c0,
                                             float inv_step) {
    if (!(x > 0.0)) return 0;
    const float l = __log2f((float)x) * 0.30102999566f;            // log10 x, FP32
    const float gf = fminf(fmaxf(floorf((l - c0) * inv_step) + 1.0f, 0.0f), (float)nthr);
    const int g = (int)gf;
    const bool lo_ok = g == 0 || st[g - 1] <= x;
    const bool hi_ok = g == nthr || x < st[g];
    return (lo_ok && hi_ok) ? g : mpd_bin(st, nthr, x);
}

__global__ void __launch_bounds__(kHistThreads) mpd_values_kernel(const double* __restrict__ mu, int64_t n,
                                                         MpdThresholds targ, const double* __restrict__ thr,
                                                         int nthr, int reps, float c0, float inv_step,
                                                         unsigned long long* __restrict__ bins) {
    extern __shared__ __align__(16) char smem[];
    double* st = reinterpret_cast<double*>(smem);
    unsigned int* sb = reinterpret_cast<unsigned int*>(st + nthr);
    const bool in_arg = nthr <= kMpdArgThr;
    for (int e = threadIdx.x; e < nthr; e += blockDim.x) st[e] = in_arg ? targ.t[e] : thr[e];
    for (int e = threadIdx.x; e < (nthr + 1) * reps; e += blockDim.x) sb[e] = 0;
    __syncthreads();
    const int r = threadIdx.x & (reps - 1);
    grid_values(mu, n, [&](double x) { atomicAdd(&sb[mpd_value_bin(st, nthr, x, c0, inv_step) * reps + r], 1u); });
    __syncthreads();
    for (int e = threadIdx.x; e <= nthr; e += blockDim.x) {
        unsigned long long t = 0;
        for (int q = 0; q < reps; ++q) t += sb[e * reps + q];
        if (t) atomicAdd(&bins[e], t);
    }
}

// Pixels with N < t_below: the host finds t_below as the first count whose
// FP64 quotient N / N_avg is not below mu_lim (the quotient is monotone in N),
// so this is the definition's decision, taken once per count value.
__global__ void __launch_bounds__(256) prob_sum_kernel(const int32_t* __restrict__ counts, int64_t n,
                                                       int64_t t_below,
                                                       unsigned long long* __restrict__ out) {
    __shared__ unsigned long long part[4];
    unsigned long long below = 0;
    grid_counts(counts, n, [&](int cv) { below += ((int64_t)cv < t_below) ? 1ull : 0ull; });
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) below += __shfl_xor(below, o);
    if ((threadIdx.x % kLanes) == 0) part[threadIdx.x / kLanes] = below;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < (int)(blockDim.x / kLanes); ++i) t += part[i];
        out[(int64_t)blockIdx.x * kRecWords] = t;
    }
}

// Mean and sample standard deviation over n_maps MPDs of one bin per thread,
// in probabilities (bin count / n_pix).
__global__ void mpd_moments_kernel(const unsigned long long* __restrict__ bins, int n_maps,
                                   int n_bins, double n_pix, double* __restrict__ mean,
                                   double* __restrict__ stdev) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_bins) return;
    double s = 0.0;
    for (int r = 0; r < n_maps; ++r) s += (double)bins[(int64_t)r * n_bins + b] / n_pix;
    const double m = s / (double)n_maps;
    double v = 0.0;
    for (int r = 0; r < n_maps; ++r) {
        const double d = (double)bins[(int64_t)r * n_bins + b] / n_pix - m;
        v += d * d;
    }
    mean[b] = m;
    stdev[b] = n_maps > 1 ? sqrt(v / (double)(n_maps - 1)) : 0.0;
}

// ----------------------------------------------------------------------------
// indexed-map codec (Appendix B)
// ----------------------------------------------------------------------------

constexpr int kScanPerBlock = 1024;   // elements per scan block (256 threads x 4)

// flag[v] = 1 where value v occurs in the map
__global__ void distinct_flag_kernel(const unsigned long long* __restrict__ hist, int64_t n,
                                     int32_t* __restrict__ flag) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        flag[v] = hist[v] ? 1 : 0;
}

// Exclusive scan of a block of 256 x 4 int32 in LDS; returns the block total.
__device__ int block_exclusive_scan_1024(int32_t (&v)[4], int* sh) {
    const int t = threadIdx.x;
    int local = v[0] + v[1] + v[2] + v[3];
    sh[t] = local;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {       // Hillis-Steele over the 256 thread sums
        const int add = t >= o ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    const int total = sh[255];
    int run = sh[t] - local;                   // exclusive prefix of this thread
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) { const int x = v[i]; v[i] = run; run += x; }
    return total;
}

__global__ void __launch_bounds__(256) scan_block_sums_kernel(const int32_t* __restrict__ in, int64_t n,
                                                              int32_t* __restrict__ sums) {
    __shared__ int sh[256];
    const int64_t base = (int64_t)blockIdx.x * kScanPerBlock + threadIdx.x * 4;
    int32_t v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = base + i < n ? in[base + i] : 0;
    const int total = block_exclusive_scan_1024(v, sh);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One workgroup: exclusive scan of the block sums in place; *grand = total.
__global__ void __launch_bounds__(256) scan_sums_kernel(int32_t* __restrict__ sums, int64_t nb,
                                                        int64_t* __restrict__ grand) {
    __shared__ int sh[256];
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += kScanPerBlock) {
        int32_t v[4];
        const int64_t base = c0 + threadIdx.x * 4;
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = base + i < nb ? sums[base + i] : 0;
        const int total = block_exclusive_scan_1024(v, sh);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (base + i < nb) sums[base + i] = (int32_t)(carry + v[i]);
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) *grand = carry;
}

__global__ void __launch_bounds__(256) scan_apply_kernel(const int32_t* __restrict__ in, int64_t n,
                                                         const int32_t* __restrict__ offsets,
                                                         int32_t* __restrict__ out) {
    __shared__ int sh[256];
    const int64_t base = (int64_t)blockIdx.x * kScanPerBlock + threadIdx.x * 4;
    int32_t v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = base + i < n ? in[base + i] : 0;
    block_exclusive_scan_1024(v, sh);
    const int32_t off = offsets[blockIdx.x];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (base + i < n) out[base + i] = off + v[i];
}

// values[rank[v]] = v for every value present (ranks ascend with v).
__global__ void scatter_values_kernel(const int32_t* __restrict__ flag,
                                      const int32_t* __restrict__ rank, int64_t n,
                                      int32_t* __restrict__ values) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        if (flag[v]) values[rank[v]] = (int32_t)v;
}

// One output word per thread for words [w_begin, n_words): gathers the
// indices of the pixels whose bits fall into word w (bits [32w, 32w + 32),
// pixel p at bits [p b, p b + b), least significant bit first). Stores are
// coalesced and need no atomics. The general path, and the tail of the
// chunked one.
__global__ void pack_kernel(const int32_t* __restrict__ counts, int64_t n_pix,
                            const int32_t* __restrict__ rank, int64_t n_values, int bits,
                            int64_t w_begin, int64_t n_words, uint32_t* __restrict__ packed) {
    for (int64_t w = w_begin + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < n_words;
         w += (int64_t)gridDim.x * blockDim.x) {
        const int64_t lo_bit = w * 32;
        const int64_t p0 = lo_bit / bits;
        int64_t p1 = (lo_bit + 31) / bits;
        if (p1 > n_pix - 1) p1 = n_pix - 1;
        unsigned long long word = 0;
        for (int64_t p = p0; p <= p1; ++p) {
            const int32_t c = counts[p];
            const unsigned long long idx =
                (c >= 0 && c < n_values) ? (unsigned long long)(uint32_t)rank[c] : 0ull;
            const int64_t start = p * bits;
            if (start >= lo_bit) word |= idx << (start - lo_bit);        // shift < 32
            else word |= idx >> (lo_bit - start);                        // shift < bits <= 32
        }
        packed[w] = (uint32_t)word;
    }
}

constexpr int kPackChunk = 4096;      // pixels per chunk: kPackChunk * bits is a whole number of words
constexpr int kPackRankLds = 8192;    // rank-table entries staged in LDS

// Chunked pack: a workgroup takes 4096 pixels at a time with coalesced
// 16-byte loads, ORs each pixel's index into an LDS word array at bit p * b
// (a multiply, no division), and stores the chunk's 128 b words coalesced.
// The rank table sits in LDS when it has at most kPackRankLds entries.
// counts 16-byte aligned; full chunks only.
template <bool LDS>
__global__ void __launch_bounds__(256) pack_chunks_kernel(const int32_t* __restrict__ counts, int64_t chunks,
                                                          const int32_t* __restrict__ rank, int64_t n_values,
                                                          int bits, uint32_t* __restrict__ packed) {
    __shared__ int32_t sr[LDS ? kPackRankLds : 1];
    __shared__ uint32_t sw[kPackChunk + 1];
    if constexpr (LDS) {
        for (int i = threadIdx.x; i < n_values; i += blockDim.x) sr[i] = rank[i];
    }
    const int nw = bits * (kPackChunk / 32);
    for (int i = threadIdx.x; i <= nw; i += blockDim.x) sw[i] = 0u;
    __syncthreads();
    for (int64_t ch = blockIdx.x; ch < chunks; ch += gridDim.x) {
        const int4* __restrict__ src = reinterpret_cast<const int4*>(counts + ch * kPackChunk);
        int4 v[kPackChunk / 1024];
#pragma unroll
        for (int u = 0; u < kPackChunk / 1024; ++u) v[u] = src[threadIdx.x + 256 * u];
#pragma unroll
        for (int u = 0; u < kPackChunk / 1024; ++u) {
            const int base = 4 * (threadIdx.x + 256 * u);
            const int c[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                uint32_t idx = 0u;
                if (c[e] >= 0 && c[e] < n_values) idx = (uint32_t)(LDS ? sr[c[e]] : rank[c[e]]);
                const int sbit = (base + e) * bits;
                const uint64_t sh = (uint64_t)idx << (sbit & 31);
                if ((uint32_t)sh) atomicOr(&sw[sbit >> 5], (uint32_t)sh);
                if ((uint32_t)(sh >> 32)) atomicOr(&sw[(sbit >> 5) + 1], (uint32_t)(sh >> 32));
            }
        }
        __syncthreads();
        uint32_t* __restrict__ dst = packed + ch * nw;
        for (int w = threadIdx.x; w < nw; w += blockDim.x) {
            dst[w] = sw[w];
            sw[w] = 0u;
        }
        if (threadIdx.x == 0) sw[nw] = 0u;
        __syncthreads();
    }
}

// Inverse of pack_kernel for pixels [p_begin, n_pix); an index past the
// table (a stream not produced by the encoder) decodes to -1 instead of
// reading out of bounds. The general path, and the tail of the 4-pixel one.
__global__ void unpack_kernel(const uint32_t* __restrict__ packed, int64_t p_begin, int64_t n_pix, int bits,
                              const int32_t* __restrict__ values, int64_t n_values,
                              int32_t* __restrict__ counts) {
    const unsigned long long mask = bits >= 32 ? 0xFFFFFFFFull : ((1ull << bits) - 1ull);
    for (int64_t p = p_begin + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n_pix;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t start = p * bits;
        const int64_t w = start >> 5;
        const int off = (int)(start & 31);
        unsigned long long v = (unsigned long long)packed[w] >> off;
        if (off + bits > 32) v |= (unsigned long long)packed[w + 1] << (32 - off);
        const unsigned long long idx = v & mask;
        counts[p] = idx < (unsigned long long)n_values ? values[idx] : -1;
    }
}

constexpr int kUnpackValuesLds = 4096;   // value-table entries staged in LDS

// 4-pixel unpack for codes of at most 16 bits: a thread decodes pixels
// 4q .. 4q + 3, whose 4 b bits lie in the three words from bit 4 q b on (read
// together before any is used; words past the stream's n_words read as 0),
// and stores them as one 16-byte write; the value table sits in LDS when it
// has at most kUnpackValuesLds entries. counts 16-byte aligned; pixels
// [0, 4 nq).
template <bool LDS>
__global__ void __launch_bounds__(256) unpack4_kernel(const uint32_t* __restrict__ packed, int64_t n_words,
                                                      int64_t nq, int bits, const int32_t* __restrict__ values,
                                                      int64_t n_values, int32_t* __restrict__ counts) {
    __shared__ int32_t sv[LDS ? kUnpackValuesLds : 1];
    if constexpr (LDS) {
        for (int i = threadIdx.x; i < n_values; i += blockDim.x) sv[i] = values[i];
        __syncthreads();
    }
    const uint32_t mask = (1u << bits) - 1u;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t start = q * 4 * bits;
        const int64_t w = start >> 5;
        const int off = (int)(start & 31);
        const uint32_t w0 = packed[w];
        const uint32_t w1 = w + 1 < n_words ? packed[w + 1] : 0u;
        const uint32_t w2 = w + 2 < n_words ? packed[w + 2] : 0u;
        const unsigned __int128 all = (unsigned __int128)w0 | ((unsigned __int128)w1 << 32) |
                                      ((unsigned __int128)w2 << 64);
        int r[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t idx = (uint32_t)(all >> (off + u * bits)) & mask;
            if constexpr (LDS) r[u] = idx < (uint32_t)n_values ? sv[idx] : -1;
            else r[u] = idx < (uint32_t)n_values ? values[idx] : -1;
        }
        reinterpret_cast<int4*>(counts)[q] = make_int4(r[0], r[1], r[2], r[3]);
    }
}

int grid_for(int64_t n, int threads, int cap) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

hipError_t launch_normalise(const int32_t* counts, int64_t n, double n_avg, float* mu,
                            hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(normalise_kernel, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, counts, n,
                       n_avg, mu);
    return hipGetLastError();
}

int reduce_blocks(int64_t n) { return grid_for(n, 256 * 16, kRedBlocks); }

hipError_t launch_count_stats(const int32_t* counts, int64_t n, const unsigned long long* escaped,
                              unsigned long long* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(count_stats_kernel, dim3(reduce_blocks(n)), dim3(256), 0, s, counts, n, escaped, out);
    return hipGetLastError();
}

hipError_t launch_count_hist(const int32_t* counts, int64_t n, int64_t n_values,
                             unsigned long long* hist, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    // fewer, longer blocks: each one zeroes and flushes its LDS histogram once
    const int reps = hist_reps(n_values < kHistLds ? n_values : kHistLds);
    hipLaunchKernelGGL(count_hist_kernel, dim3(grid_for(n, kHistThreads * 16, kHistBlocks)), dim3(kHistThreads),
                       (size_t)kHistLds * sizeof(unsigned int), s, counts, n, n_values, reps, hist);
    return hipGetLastError();
}

hipError_t launch_mpd(const int32_t* counts, int64_t n, const MpdThresholds& args, const double* thr,
                      int nthr, unsigned long long* bins, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    // the copies get what the thresholds and the table leave of 64 KiB, at most kHistLds words
    const int64_t fixed = (int64_t)nthr * (int64_t)sizeof(double) + (int64_t)kMpdLut * (int64_t)sizeof(uint16_t);
    const int64_t spare = (65536 - fixed) / (int64_t)sizeof(unsigned int);
    const int reps = hist_reps(nthr + 1, spare < kHistLds ? spare : kHistLds);
    const size_t lds = (size_t)nthr * sizeof(double) + (size_t)(nthr + 1) * reps * sizeof(unsigned int) +
                       (size_t)kMpdLut * sizeof(uint16_t);
    hipLaunchKernelGGL(mpd_kernel, dim3(grid_for(n, kHistThreads * 16, kHistBlocks)), dim3(kHistThreads), lds, s,
                       counts, n, args, thr, nthr, reps, bins);
    return hipGetLastError();
}

hipError_t launch_mpd_values(const double* mu, int64_t n, const MpdThresholds& args, const double* thr,
                             int nthr, float c0, float inv_step, unsigned long long* bins, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t fixed = (int64_t)nthr * (int64_t)sizeof(double);
    const int64_t spare = (65536 - fixed) / (int64_t)sizeof(unsigned int);
    const int reps = hist_reps(nthr + 1, spare < kHistLds ? spare : kHistLds);
    const size_t lds = (size_t)nthr * sizeof(double) + (size_t)(nthr + 1) * reps * sizeof(unsigned int);
    hipLaunchKernelGGL(mpd_values_kernel, dim3(grid_for(n, kHistThreads * 8, kHistBlocks)), dim3(kHistThreads), lds,
                       s, mu, n, args, thr, nthr, reps, c0, inv_step, bins);
    return hipGetLastError();
}

hipError_t launch_prob_sum(const int32_t* counts, int64_t n, int64_t t_below,
                           unsigned long long* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(prob_sum_kernel, dim3(reduce_blocks(n)), dim3(256), 0, s, counts, n, t_below, out);
    return hipGetLastError();
}

hipError_t launch_mpd_moments(const unsigned long long* bins, int n_maps, int n_bins, double n_pix,
                              double* mean, double* stdev, hipStream_t s) {
    if (n_bins <= 0) return hipSuccess;
    hipLaunchKernelGGL(mpd_moments_kernel, dim3((n_bins + 255) / 256), dim3(256), 0, s, bins, n_maps,
                       n_bins, n_pix, mean, stdev);
    return hipGetLastError();
}

int64_t scan_blocks(int64_t n) { return (n + kScanPerBlock - 1) / kScanPerBlock; }

hipError_t launch_distinct_ranks(const unsigned long long* hist, int64_t n_values, int32_t* flag,
                                 int32_t* rank, int32_t* block_sums, int64_t* total,
                                 hipStream_t s) {
    if (n_values <= 0) return hipSuccess;
    const int64_t nb = scan_blocks(n_values);
    hipLaunchKernelGGL(distinct_flag_kernel, dim3(grid_for(n_values, 256, 8192)), dim3(256), 0, s, hist,
                       n_values, flag);
    hipLaunchKernelGGL(scan_block_sums_kernel, dim3((unsigned)nb), dim3(256), 0, s, flag, n_values,
                       block_sums);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(256), 0, s, block_sums, nb, total);
    hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(256), 0, s, flag, n_values,
                       block_sums, rank);
    return hipGetLastError();
}

hipError_t launch_codec_pack(const int32_t* counts, int64_t n_pix, const int32_t* flag,
                             const int32_t* rank, int64_t n_values, int bits, int32_t* values,
                             uint32_t* packed, hipStream_t s) {
    const int64_t n_words = (n_pix * bits + 31) / 32;
    hipLaunchKernelGGL(scatter_values_kernel, dim3(grid_for(n_values, 256, 8192)), dim3(256), 0, s, flag,
                       rank, n_values, values);
    // whole 4096-pixel chunks through the chunked kernel when the counts are
    // 16-byte aligned, the remaining words word by word
    const int64_t chunks = (reinterpret_cast<uintptr_t>(counts) % 16 == 0) ? n_pix / kPackChunk : 0;
    if (chunks > 0) {
        const int g = grid_for(chunks, 1, 2048);
        if (n_values <= kPackRankLds)
            hipLaunchKernelGGL(pack_chunks_kernel<true>, dim3(g), dim3(256), 0, s, counts, chunks, rank,
                               n_values, bits, packed);
        else
            hipLaunchKernelGGL(pack_chunks_kernel<false>, dim3(g), dim3(256), 0, s, counts, chunks, rank,
                               n_values, bits, packed);
    }
    const int64_t w_begin = chunks * (kPackChunk / 32) * bits;
    if (w_begin < n_words)
        hipLaunchKernelGGL(pack_kernel, dim3(grid_for(n_words - w_begin, 256, 16384)), dim3(256), 0, s,
                           counts, n_pix, rank, n_values, bits, w_begin, n_words, packed);
    return hipGetLastError();
}

hipError_t launch_codec_unpack(const uint32_t* packed, int64_t n_pix, int bits, const int32_t* values,
                               int64_t n_values, int32_t* counts, hipStream_t s) {
    if (n_pix <= 0) return hipSuccess;
    // 4 pixels per thread for codes of <= 16 bits into 16-byte aligned maps;
    // the last n_pix % 4 pixels (or all, otherwise) one per thread
    const int64_t nq = (bits <= 16 && reinterpret_cast<uintptr_t>(counts) % 16 == 0) ? n_pix / 4 : 0;
    if (nq > 0) {
        const int g = grid_for(nq, 256, 2048);
        const int64_t n_words = (n_pix * bits + 31) / 32;
        if (n_values <= kUnpackValuesLds)
            hipLaunchKernelGGL(unpack4_kernel<true>, dim3(g), dim3(256), 0, s, packed, n_words, nq, bits,
                               values, n_values, counts);
        else
            hipLaunchKernelGGL(unpack4_kernel<false>, dim3(g), dim3(256), 0, s, packed, n_words, nq, bits,
                               values, n_values, counts);
    }
    if (4 * nq < n_pix)
        hipLaunchKernelGGL(unpack_kernel, dim3(grid_for(n_pix - 4 * nq, 256, 16384)), dim3(256), 0, s,
                           packed, 4 * nq, n_pix, bits, values, n_values, counts);
    return hipGetLastError();
}

}  // namespace rl
