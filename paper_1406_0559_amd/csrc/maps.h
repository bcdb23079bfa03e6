// Internal declarations of the kernels on finished maps (maps.hip: statistics,
// MPDs, probability sums, codec) and of the finite-source convolution
// (convolve.hip), for the C-ABI layer. Not part of the public interface.
#pragma once

#include "internal.h"

namespace rl {

// Launchers; each returns the hipError_t of the launch.
hipError_t launch_normalise(const int32_t* counts, int64_t n, double n_avg, float* mu,
                            hipStream_t stream);
// Scalar reductions over a map (count statistics, probability sums): each
// workgroup stores one record of kRecWords u64 words at out[kRecWords * b]
// (no atomics, so nothing has to be zeroed first), reduce_blocks(n) records
// in all, and the host folds them. `out` may be device-mapped pinned host
// memory, so that the records need no copy before the host reads them.
constexpr int kRedBlocks = 2048;
constexpr int kRecWords = 4;
constexpr size_t kRedBytes = (size_t)kRedBlocks * kRecWords * sizeof(unsigned long long);
int reduce_blocks(int64_t n);
// record: word 0 sums the non-negative counts, word 1 is the largest count,
// word 2 counts the negative ones; with `escaped` non-null, workgroup 0 also
// copies *escaped to out[kRedBlocks * kRecWords]
hipError_t launch_count_stats(const int32_t* counts, int64_t n, const unsigned long long* escaped,
                              unsigned long long* out, hipStream_t stream);
hipError_t launch_count_hist(const int32_t* counts, int64_t n, int64_t n_values,
                             unsigned long long* hist, hipStream_t stream);
// Thresholds of at most kMpdArgThr entries travel as a kernel argument (no
// copy ahead of the launch); longer lists are read from thr in device memory.
constexpr int kMpdArgThr = 256;
struct MpdThresholds {
    double t[kMpdArgThr];
};
hipError_t launch_mpd(const int32_t* counts, int64_t n, const MpdThresholds& args, const double* thr,
                      int nthr, unsigned long long* bins, hipStream_t stream);
// The same binning of a map of real magnifications (thresholds mu_ref 10^edge);
// c0 = log10 mu_ref + log_lo and inv_step = nbins / (log_hi - log_lo) only
// guide the search (a guessed bin is kept if the thresholds confirm it).
hipError_t launch_mpd_values(const double* mu, int64_t n, const MpdThresholds& args, const double* thr,
                             int nthr, float c0, float inv_step, unsigned long long* bins, hipStream_t stream);
// record word 0 counts the pixels below t_below
hipError_t launch_prob_sum(const int32_t* counts, int64_t n, int64_t t_below,
                           unsigned long long* out, hipStream_t s);
hipError_t launch_mpd_moments(const unsigned long long* bins, int n_maps, int n_bins, double n_pix,
                              double* mean, double* stdev, hipStream_t stream);

constexpr int kMaxMpdBins = 4096;
constexpr int kMpdLut = 4096;   // count values binned through a table

// Indexed-map codec: flag/rank the distinct values of a count histogram
// (exclusive scan; *total = number of distinct values), then pack / unpack.
int64_t scan_blocks(int64_t n);
hipError_t launch_distinct_ranks(const unsigned long long* hist, int64_t n_values, int32_t* flag,
                                 int32_t* rank, int32_t* block_sums, int64_t* total,
                                 hipStream_t stream);
hipError_t launch_codec_pack(const int32_t* counts, int64_t n_pix, const int32_t* flag,
                             const int32_t* rank, int64_t n_values, int bits, int32_t* values,
                             uint32_t* packed, hipStream_t stream);
hipError_t launch_codec_unpack(const uint32_t* packed, int64_t n_pix, int bits, const int32_t* values,
                               int64_t n_values, int32_t* counts, hipStream_t stream);

// Finite-source convolution (convolve.hip). Sides: products of 2, 3 and 5 in
// [2, kMaxFftSide].
bool fft_side_supported(int n);
size_t convolve_scratch_bytes(int p1, int p2);
// The map is convolved with kernels[0 .. n) into outs[0 .. n) (host arrays
// of device pointers). The scratch holds the stage-twiddle tables of both
// axes at offsets fixed by (p1, p2); twiddles_ready says that a previous call
// with the same sides and the same scratch buffer left them there (and what
// else the power-of-two path keeps with them), so they are not recomputed.
hipError_t launch_convolve(const int32_t* counts, const double* const* kernels, int n, int p1, int p2,
                           double n_avg, double* const* outs, void* scratch, bool twiddles_ready,
                           hipStream_t stream);
size_t source_scratch_bytes(int h1, int h2);
hipError_t launch_source_kernel(int shape, double radius, double hole, double pix1, double pix2,
                                int h1, int h2, int p1, int p2, double* kernel, double* scratch,
                                hipStream_t stream);
size_t table_data_offset(int nx, int ny, int h1, int h2);
size_t table_scratch_bytes(int nx, int ny, int h1, int h2);
hipError_t launch_table_kernel(int nx, int ny, double pix1, double pix2, int h1, int h2, int p1, int p2,
                               double* kernel, void* scratch, hipStream_t stream);
constexpr int kMaxFftSide = 10240;

}  // namespace rl
