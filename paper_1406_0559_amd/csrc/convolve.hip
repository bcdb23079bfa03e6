// Finite-source maps on gfx950: a map convolved with a source profile
// (Vernardos & Fluke 2014, Section 2.4, eq. 6: C = F^-1[F(M) F(K)]).
//
// The kernel K is the source profile binned at the map's pixel size, centred
// on pixel (0, 0) with wrap-around and normalised to unit sum. Both the map M
// (integer counts) and K are real, so one complex 2D FFT of Z = M + iK gives
// both spectra (F(M)[u] = (Z[u] + conj Z[-u]) / 2, F(K)[u] = (Z[u] - conj Z[-u]) / 2i);
// their product is Hermitian, and one inverse 2D FFT returns C. All in FP64.
//
// 2D FFTs are row FFTs (one workgroup per row, radix-2 in LDS with a
// bit-reversed load), a tiled transpose, and row FFTs again; the product is
// formed in the transposed layout and the inverse undoes the two passes in
// reverse order. Sizes are powers of two up to 4096 per side (a 4096-point
// complex FP64 row is the 64 KiB of LDS one workgroup may use).
#include <climits>

#include "internal.h"

namespace rl {
namespace {

struct cplx { double x, y; };

__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
    return cplx{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// tw[k] = exp(-2 pi i k / n), k < n / 2
__global__ void twiddle_kernel(cplx* __restrict__ tw, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n / 2) return;
    double s, c;
    sincospi(2.0 * (double)k / (double)n, &s, &c);
    tw[k] = cplx{c, -s};
}

__global__ void pack_kernel(const int32_t* __restrict__ m, const double* __restrict__ k, int64_t n,
                            cplx* __restrict__ z) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        z[i] = cplx{(double)m[i], k[i]};
}

// In-place FFT of each row of length n = 2^logn (one workgroup per row).
// Forward uses tw, inverse its conjugate; no scaling.
__global__ void __launch_bounds__(256) fft_rows_kernel(cplx* __restrict__ z, int n, int logn,
                                                       const cplx* __restrict__ tw, int inverse) {
    extern __shared__ __align__(16) char smem[];
    cplx* buf = reinterpret_cast<cplx*>(smem);
    cplx* row = z + (int64_t)blockIdx.x * n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int r = (int)(__brev((unsigned)i) >> (32 - logn));
        buf[r] = row[i];
    }
    __syncthreads();
    for (int half = 1; half < n; half <<= 1) {
        const int stride = n / (2 * half);
        for (int b = threadIdx.x; b < n / 2; b += blockDim.x) {
            const int j = b & (half - 1);
            const int i0 = ((b - j) << 1) + j;
            const int i1 = i0 + half;
            cplx w = tw[j * stride];
            if (inverse) w.y = -w.y;
            const cplx t = cmul(w, buf[i1]);
            const cplx a = buf[i0];
            buf[i0] = cplx{a.x + t.x, a.y + t.y};
            buf[i1] = cplx{a.x - t.x, a.y - t.y};
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) row[i] = buf[i];
}

// out (cols x rows) = transpose of in (rows x cols), 32 x 32 tiles via LDS.
__global__ void __launch_bounds__(256) transpose_kernel(const cplx* __restrict__ in, cplx* __restrict__ out,
                                                        int rows, int cols) {
    __shared__ cplx tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;   // 32 x 8 threads
    for (int j = ty; j < 32; j += 8) {
        const int r = by + j, c = bx + tx;
        if (r < rows && c < cols) tile[j][tx] = in[(int64_t)r * cols + c];
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        const int r = bx + j, c = by + tx;       // out row = in column
        if (r < cols && c < rows) out[(int64_t)r * rows + c] = tile[tx][j];
    }
}

// Spectrum product in the transposed layout t (n1 rows of length n2, entry
// (u1, u2) = Z-hat(u2, u1)): each pair (u, -u) is handled by one thread.
__global__ void product_kernel(cplx* __restrict__ t, int n1, int n2) {
    const int64_t total = (int64_t)n1 * n2;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int u1 = (int)(i / n2), u2 = (int)(i % n2);
        const int64_t p = (int64_t)((n1 - u1) % n1) * n2 + (n2 - u2) % n2;
        if (p < i) continue;
        const cplx zu = t[i], zm = t[p];
        // F(M)[u] = (zu + conj zm) / 2, F(K)[u] = (zu - conj zm) / (2i)
        const cplx fm = cplx{0.5 * (zu.x + zm.x), 0.5 * (zu.y - zm.y)};
        const cplx dk = cplx{zu.x - zm.x, zu.y + zm.y};
        const cplx fk = cplx{0.5 * dk.y, -0.5 * dk.x};
        const cplx prod = cmul(fm, fk);
        t[i] = prod;
        if (p != i) t[p] = cplx{prod.x, -prod.y};
    }
}

__global__ void output_kernel(const cplx* __restrict__ z, int64_t n, double scale,
                              double* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = z[i].x * scale;
}

// ----------------------------------------------------------------------------
// source kernels
// ----------------------------------------------------------------------------

__device__ double brightness(int shape, double r, double radius, double hole) {
    if (!(r < radius) || r < hole) return 0.0;
    if (shape == 0) return 1.0;
    if (shape == 1) {
        const double sigma = radius / 3.0;
        return exp(-(r * r) / (2.0 * sigma * sigma));
    }
    const double core = radius / 100.0;
    return pow((r > core ? r : core) / radius, -0.75);
}

// Pixel (i, j), |i| <= h1, |j| <= h2, gets the mean brightness over an s x s
// grid of sub-samples, stored compactly at q = (j + h2) (2 h1 + 1) + (i + h1).
__global__ void source_samples_kernel(int shape, double radius, double hole, double pix1, double pix2,
                                      int h1, int h2, int s, double* __restrict__ compact) {
    const int w = 2 * h1 + 1;
    const int64_t total = (int64_t)w * (2 * h2 + 1);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(q % w) - h1, j = (int)(q / w) - h2;
        double acc = 0.0;
        for (int b = 0; b < s; ++b) {
            const double y = ((double)j + (((double)b + 0.5) / (double)s - 0.5)) * pix2;
            for (int a = 0; a < s; ++a) {
                const double x = ((double)i + (((double)a + 0.5) / (double)s - 0.5)) * pix1;
                acc += brightness(shape, hypot(x, y), radius, hole);
            }
        }
        compact[q] = acc / (double)(s * s);
    }
}

// One workgroup, fixed summation order: the normalisation is reproducible.
__global__ void __launch_bounds__(256) ordered_sum_kernel(const double* __restrict__ v, int64_t n,
                                                          double* __restrict__ out) {
    __shared__ double part[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += v[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < (int)blockDim.x; ++i) t += part[i];
        *out = t;
    }
}

// kernel[(j mod p2), (i mod p1)] = compact[q] / total
__global__ void scatter_kernel(const double* __restrict__ compact, int h1, int h2, int p1, int p2,
                               const double* __restrict__ total, double* __restrict__ k) {
    const int w = 2 * h1 + 1;
    const int64_t m = (int64_t)w * (2 * h2 + 1);
    const double t = *total;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < m;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(q % w) - h1, j = (int)(q / w) - h2;
        const int ii = ((i % p1) + p1) % p1, jj = ((j % p2) + p2) % p2;
        k[(int64_t)jj * p1 + ii] = compact[q] / t;
    }
}

__global__ void zero_f64_kernel(double* __restrict__ v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        v[i] = 0.0;
}

int grid_of(int64_t n, int cap) {
    int64_t g = (n + 255) / 256;
    return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

int log2i(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

hipError_t fft_rows(cplx* z, int rows, int n, const cplx* tw, bool inverse, hipStream_t s) {
    hipLaunchKernelGGL(fft_rows_kernel, dim3(rows), dim3(256), (size_t)n * sizeof(cplx), s, z, n,
                       log2i(n), tw, inverse ? 1 : 0);
    return hipGetLastError();
}

hipError_t transpose(const cplx* in, cplx* out, int rows, int cols, hipStream_t s) {
    hipLaunchKernelGGL(transpose_kernel, dim3((cols + 31) / 32, (rows + 31) / 32), dim3(256), 0, s, in,
                       out, rows, cols);
    return hipGetLastError();
}

}  // namespace

size_t convolve_scratch_bytes(int p1, int p2) {
    const size_t plane = (size_t)p1 * p2 * sizeof(cplx);
    return 2 * plane + (size_t)(p1 / 2 + p2 / 2 + 2) * sizeof(cplx) + 256;
}

hipError_t launch_convolve(const int32_t* counts, const double* kernel, int p1, int p2, double n_avg,
                           double* out, void* scratch, hipStream_t s) {
    const int64_t n = (int64_t)p1 * p2;
    cplx* z = static_cast<cplx*>(scratch);              // p2 x p1
    cplx* t = z + n;                                    // p1 x p2
    cplx* tw1 = t + n;                                  // p1 / 2 twiddles
    cplx* tw2 = tw1 + (p1 / 2 > 0 ? p1 / 2 : 1);        // p2 / 2 twiddles
    hipLaunchKernelGGL(twiddle_kernel, dim3((p1 / 2 + 255) / 256 + 1), dim3(256), 0, s, tw1, p1);
    hipLaunchKernelGGL(twiddle_kernel, dim3((p2 / 2 + 255) / 256 + 1), dim3(256), 0, s, tw2, p2);
    hipLaunchKernelGGL(pack_kernel, dim3(grid_of(n, 8192)), dim3(256), 0, s, counts, kernel, n, z);
    hipError_t e = fft_rows(z, p2, p1, tw1, false, s);           // along x1
    if (e == hipSuccess) e = transpose(z, t, p2, p1, s);         // t: p1 x p2
    if (e == hipSuccess) e = fft_rows(t, p1, p2, tw2, false, s); // along x2
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(product_kernel, dim3(grid_of(n, 8192)), dim3(256), 0, s, t, p1, p2);
    e = fft_rows(t, p1, p2, tw2, true, s);
    if (e == hipSuccess) e = transpose(t, z, p1, p2, s);
    if (e == hipSuccess) e = fft_rows(z, p2, p1, tw1, true, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(output_kernel, dim3(grid_of(n, 8192)), dim3(256), 0, s, z, n,
                       1.0 / ((double)n * n_avg), out);
    return hipGetLastError();
}

size_t source_scratch_bytes(int h1, int h2) {
    return ((size_t)(2 * h1 + 1) * (2 * h2 + 1) + 2) * sizeof(double) + 256;
}

hipError_t launch_source_kernel(int shape, double radius, double hole, double pix1, double pix2,
                                int h1, int h2, int p1, int p2, double* kernel, double* scratch,
                                hipStream_t s) {
    const int64_t n = (int64_t)p1 * p2;
    const int64_t m = (int64_t)(2 * h1 + 1) * (2 * h2 + 1);
    double* total = scratch;
    double* compact = scratch + 2;
    hipLaunchKernelGGL(zero_f64_kernel, dim3(grid_of(n, 8192)), dim3(256), 0, s, kernel, n);
    hipLaunchKernelGGL(source_samples_kernel, dim3(grid_of(m, 8192)), dim3(256), 0, s, shape, radius,
                       hole, pix1, pix2, h1, h2, 8, compact);
    hipLaunchKernelGGL(ordered_sum_kernel, dim3(1), dim3(256), 0, s, compact, m, total);
    hipLaunchKernelGGL(scatter_kernel, dim3(grid_of(m, 8192)), dim3(256), 0, s, compact, h1, h2, p1, p2,
                       total, kernel);
    return hipGetLastError();
}

}  // namespace rl
