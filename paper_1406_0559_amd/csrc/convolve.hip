// Finite-source maps on gfx950: a map convolved with a source profile
// (Vernardos & Fluke 2014, Section 2.4, eq. 6: C = F^-1[F(M) F(K)]).
//
// The kernel K is the source profile binned at the map's pixel size, centred
// on pixel (0, 0) with wrap-around and normalised to unit sum. Both the map M
// (integer counts) and K are real, so one complex 2D FFT of Z = M + iK gives
// both spectra (F(M)[u] = (Z[u] + conj Z[-u]) / 2, F(K)[u] = (Z[u] - conj Z[-u]) / 2i);
// their product is Hermitian, and one inverse 2D FFT returns C. All in FP64.
//
// K is scaled by a power of two before packing so that both spectra keep full
// precision (see norms_kernel). Each axis is a batch of row FFTs in LDS, one
// workgroup per row: mixed radix (16, 8, 4, 2, 3, 5), decimation in time from a
// digit-reversed load for forward transforms and decimation in frequency with
// a digit-reversed store for inverse ones, so no pass needs a separate
// reordering. After a norm reduction, five passes over HBM:
//   1. forward along x1, packing Z = M + i 2^e K on load;
//   2. transpose (32 x 32 LDS tiles);
//   3. per pair of rows u1, -u1: forward along x2, spectrum product, inverse
//      along x2 (the pair shares one workgroup, so the product needs no pass);
//   4. transpose back;
//   5. inverse along x1, writing Re(C) / (p1 p2 n_avg).
// Sides are products of 2, 3 and 5 up to 10240 (one FP64 complex row of 10240
// points is 160 KiB, the LDS of one workgroup on gfx950); sides above 5120 do
// pass 3 as forward rows, a product pass and inverse rows.
#include <climits>

#include "maps.h"

namespace rl {
namespace {

struct cplx { double x, y; };

__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
    return cplx{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return cplx{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return cplx{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cplx cscale(cplx a, double s) { return cplx{a.x * s, a.y * s}; }
__device__ __forceinline__ cplx conj(cplx a) { return cplx{a.x, -a.y}; }
// sg * i * a, sg = +1 or -1
__device__ __forceinline__ cplx rot(cplx a, double sg) { return cplx{-sg * a.y, sg * a.x}; }


// In-place DFTs of 2, 3, 4, 5, 8, 10 and 16 points:
// y_k = sum_q a_q exp(sg 2 pi i k q / r), sg = -1 forward, +1 inverse.
constexpr double kSin60 = 0.86602540378443864676;    // sqrt(3) / 2
constexpr double kCos72 = 0.30901699437494742410;    // (sqrt(5) - 1) / 4
constexpr double kCos144 = -0.80901699437494742410;  // -(sqrt(5) + 1) / 4
constexpr double kSin72 = 0.95105651629515357212;
constexpr double kSin144 = 0.58778525229247312917;

// cos and sin of 2 pi m / 10, m = 0 .. 9
constexpr double kC10[10] = {1.0, 0.80901699437494742410, 0.30901699437494742410,
                             -0.30901699437494742410, -0.80901699437494742410, -1.0,
                             -0.80901699437494742410, -0.30901699437494742410,
                             0.30901699437494742410, 0.80901699437494742410};
constexpr double kS10[10] = {0.0, 0.58778525229247312917, 0.95105651629515357212,
                             0.95105651629515357212, 0.58778525229247312917, 0.0,
                             -0.58778525229247312917, -0.95105651629515357212,
                             -0.95105651629515357212, -0.58778525229247312917};

// cos and sin of 2 pi m / 16, m = 0 .. 15
constexpr double kC16[16] = {1.0, 0.92387953251128675613, 0.70710678118654752440,
                             0.38268343236508977173, 0.0, -0.38268343236508977173,
                             -0.70710678118654752440, -0.92387953251128675613, -1.0,
                             -0.92387953251128675613, -0.70710678118654752440,
                             -0.38268343236508977173, 0.0, 0.38268343236508977173,
                             0.70710678118654752440, 0.92387953251128675613};
constexpr double kS16[16] = {0.0, 0.38268343236508977173, 0.70710678118654752440,
                             0.92387953251128675613, 1.0, 0.92387953251128675613,
                             0.70710678118654752440, 0.38268343236508977173, 0.0,
                             -0.38268343236508977173, -0.70710678118654752440,
                             -0.92387953251128675613, -1.0, -0.92387953251128675613,
                             -0.70710678118654752440, -0.38268343236508977173};

template <int R>
__device__ __forceinline__ void small_dft(cplx* a, double sg);

// DFT of R = A B points as A-point DFTs, twiddles exp(sg 2 pi i q2 k1 / R) and
// B-point DFTs: with q = B q1 + q2 and k = k1 + A k2,
// y_k = sum_q2 w_R^(q2 k1) w_B^(q2 k2) sum_q1 a_(B q1 + q2) w_A^(q1 k1).
template <int A, int B>
__device__ __forceinline__ void composite_dft(cplx* a, double sg) {
    constexpr int R = A * B;
    cplx t[B][A];
#pragma unroll
    for (int q2 = 0; q2 < B; ++q2) {
#pragma unroll
        for (int q1 = 0; q1 < A; ++q1) t[q2][q1] = a[B * q1 + q2];
        small_dft<A>(t[q2], sg);
#pragma unroll
        for (int k1 = 1; k1 < A; ++k1) {
            if (q2 == 0) continue;
            cplx w;
            if constexpr (16 % R == 0) {
                const int m = ((q2 * k1) % R) * (16 / R);   // index into the 16th roots
                w = cplx{kC16[m], sg * kS16[m]};
            } else {
                static_assert(R == 10, "composite DFTs of 16 / 8 or 10 points");
                const int m = (q2 * k1) % 10;
                w = cplx{kC10[m], sg * kS10[m]};
            }
            t[q2][k1] = cmul(t[q2][k1], w);
        }
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
        cplx u[B];
#pragma unroll
        for (int q2 = 0; q2 < B; ++q2) u[q2] = t[q2][k1];
        small_dft<B>(u, sg);
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) a[k1 + A * k2] = u[k2];
    }
}

template <int R>
__device__ __forceinline__ void small_dft(cplx* a, double sg) {
    if constexpr (R == 16) {
        composite_dft<4, 4>(a, sg);
    } else if constexpr (R == 10) {
        composite_dft<5, 2>(a, sg);
    } else if constexpr (R == 8) {
        composite_dft<4, 2>(a, sg);
    } else if constexpr (R == 2) {
        const cplx t = a[1];
        a[1] = csub(a[0], t);
        a[0] = cadd(a[0], t);
    } else if constexpr (R == 3) {
        const cplx t = cadd(a[1], a[2]);
        const cplx d = cscale(csub(a[1], a[2]), kSin60);
        const cplx m = csub(a[0], cscale(t, 0.5));
        a[0] = cadd(a[0], t);
        a[1] = cadd(m, rot(d, sg));
        a[2] = csub(m, rot(d, sg));
    } else if constexpr (R == 4) {
        const cplx t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
        const cplx t2 = cadd(a[1], a[3]), t3 = rot(csub(a[1], a[3]), sg);
        a[0] = cadd(t0, t2);
        a[2] = csub(t0, t2);
        a[1] = cadd(t1, t3);
        a[3] = csub(t1, t3);
    } else {
        const cplx t1 = cadd(a[1], a[4]), t2 = cadd(a[2], a[3]);
        const cplx d1 = csub(a[1], a[4]), d2 = csub(a[2], a[3]);
        const cplx p1 = cadd(a[0], cadd(cscale(t1, kCos72), cscale(t2, kCos144)));
        const cplx p2 = cadd(a[0], cadd(cscale(t1, kCos144), cscale(t2, kCos72)));
        const cplx q1 = rot(cadd(cscale(d1, kSin72), cscale(d2, kSin144)), sg);
        const cplx q2 = rot(csub(cscale(d1, kSin144), cscale(d2, kSin72)), sg);
        a[0] = cadd(a[0], cadd(t1, t2));
        a[1] = cadd(p1, q1);
        a[4] = csub(p1, q1);
        a[2] = cadd(p2, q2);
        a[3] = csub(p2, q2);
    }
}

}  // namespace

// Mixed-radix plan of one FFT length n = r_0 r_1 ... r_{ns-1} (radices 16, 8,
// 4, 2, 3, 5: the fewest LDS passes for powers of two).
// L[s] = r_0 ... r_{s-1}; stage s joins n / L[s+1] groups of r_s transforms of
// length L[s]. For L[s] > 1, div[s] = ceil(2^32 / L[s]) divides a butterfly
// index by L[s] with one high multiply (exact for index * L[s] < 2^32).
struct FftPlan {
    int32_t n, ns;
    int32_t r[16];
    int32_t L[17];
    uint32_t div[16];
};

namespace {

// max_pow2: the largest power-of-two radix to use (16, 8, 4 or 2), chosen so
// that every thread of the workgroup has a butterfly in each stage.
bool make_plan(int n, FftPlan* P, int max_pow2 = 16) {
    if (n < 2) return false;
    P->n = n;
    P->ns = 0;
    int m = n;
    auto push = [&](int r) {
        if (P->ns >= 16) return false;
        P->r[P->ns++] = r;
        m /= r;
        return true;
    };
    // powers of two: as many max_pow2 stages as fit, the remainder folded in
    // so that a radix-2 stage is left only when nothing larger fits
    int e = 0;
    while (m % 2 == 0) { m /= 2; ++e; }
    m = n;
    const int k = max_pow2 >= 16 ? 4 : (max_pow2 >= 8 ? 3 : 2);
    const int q = e / k, rem = e % k;
    for (int i = 0; i < q; ++i) {
        // the last full stage absorbs a single leftover factor 2 (R 2 = R/2 4)
        const bool split = rem == 1 && i == q - 1 && k > 2;
        if (split) {
            if (!push(1 << (k - 1)) || !push(4)) return false;
        } else if (!push(1 << k)) {
            return false;
        }
    }
    if (rem == 1 && (q == 0 || k == 2)) { if (!push(2)) return false; }
    if (rem == 2) { if (!push(4)) return false; }
    if (rem == 3) { if (!push(8)) return false; }
    while (m % 3 == 0) if (!push(3)) return false;
    while (m % 5 == 0) if (!push(5)) return false;
    if (m != 1) return false;
    P->L[0] = 1;
    for (int s = 0; s < P->ns; ++s) {
        P->L[s + 1] = P->L[s] * P->r[s];
        P->div[s] = P->L[s] == 1 ? 0u
                  : (uint32_t)((((uint64_t)1 << 32) + (uint64_t)P->L[s] - 1) / (uint64_t)P->L[s]);
    }
    return true;
}

// Position of natural index i in the digit-reversed order that an in-place
// decimation-in-time pass reads (and a decimation-in-frequency pass writes).
__device__ __forceinline__ int digit_pos(int i, const FftPlan& P) {
    int p = 0;
    for (int s = P.ns - 1; s >= 0; --s) {
        int d;
        switch (P.r[s]) {
            case 16: d = i & 15; i >>= 4; break;
            case 8: d = i & 7; i >>= 3; break;
            case 4: d = i & 3; i >>= 2; break;
            case 2: d = i & 1; i >>= 1; break;
            case 3: d = i % 3; i /= 3; break;
            default: d = i % 5; i /= 5; break;
        }
        p += d * P.L[s];
    }
    return p;
}

// LDS slot of element e of a row: the low four bits are XORed with the higher
// nibbles, a bijection inside every 16-element block (16 complex doubles are
// the 256 bytes of one pass over the 64 banks). Digit-reversed loads and the
// first stages access elements at large power-of-two strides, which would
// otherwise land on the same banks. Rows are padded to multiples of 16, so
// the slot stays inside the row's region.
__device__ __forceinline__ int swz(int e) { return e ^ (((e >> 4) ^ (e >> 8) ^ (e >> 12)) & 15); }

// Twiddles in stage order: stage s stores w^(j q) = exp(-2 pi i j q / L[s+1])
// for j < L[s], q = 1 .. r_s - 1 at tw[(L[s] - 1) + j (r_s - 1) + q - 1], so the
// butterflies of consecutive j read consecutive entries. The stages hold
// sum_s L[s] (r_s - 1) = n - 1 entries.
__global__ void stage_twiddle_kernel(cplx* __restrict__ tw, FftPlan P) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P.n - 1) return;
    int s = 0;
    while (s + 1 < P.ns && e >= P.L[s + 1] - 1) ++s;
    const int local = e - (P.L[s] - 1);
    const int r1 = P.r[s] - 1;
    const int j = local / r1, q = local - j * r1 + 1;
    double sn, cs;
    sincospi(2.0 * (double)((int64_t)j * q) / (double)P.L[s + 1], &sn, &cs);
    tw[e] = cplx{cs, -sn};
}

// One stage over `rows` LDS rows of length n, ld elements apart. DIT: twiddle,
// then DFT; DIF: DFT, then twiddle; tw is the plan's stage-ordered twiddle
// table, conjugated for the inverse.
template <int R, bool DIF>
__device__ __forceinline__ void stage(cplx* buf, const FftPlan& P, int s, int rows, int ld,
                                      const cplx* __restrict__ tw, bool inverse) {
    const int n = P.n, Ls = P.L[s], Ln = P.L[s + 1];
    const int nb = n / R;
    const cplx* __restrict__ tws = tw + (Ls - 1);
    const double sg = inverse ? 1.0 : -1.0;
    for (int b = threadIdx.x; b < rows * nb; b += blockDim.x) {
        int bb = b, row = 0;
        while (bb >= nb) { bb -= nb; ++row; }
        const int g = Ls == 1 ? bb : (int)__umulhi((unsigned)bb, P.div[s]);
        const int j = bb - g * Ls;
        cplx* rb = buf + row * ld;
        const int e0 = g * Ln + j;
        cplx a[R];
#pragma unroll
        for (int q = 0; q < R; ++q) a[q] = rb[swz(e0 + q * Ls)];
        if (!DIF) {
#pragma unroll
            for (int q = 1; q < R; ++q) {
                cplx w = tws[j * (R - 1) + q - 1];
                if (inverse) w.y = -w.y;
                a[q] = cmul(a[q], w);
            }
        }
        small_dft<R>(a, sg);
        if (DIF) {
#pragma unroll
            for (int q = 1; q < R; ++q) {
                cplx w = tws[j * (R - 1) + q - 1];
                if (inverse) w.y = -w.y;
                a[q] = cmul(a[q], w);
            }
        }
#pragma unroll
        for (int q = 0; q < R; ++q) rb[swz(e0 + q * Ls)] = a[q];
    }
}

template <bool DIF>
__device__ void run_stage(cplx* buf, const FftPlan& P, int s, int rows, int ld, const cplx* tw,
                          bool inverse) {
    switch (P.r[s]) {
        case 16: stage<16, DIF>(buf, P, s, rows, ld, tw, inverse); break;
        case 8: stage<8, DIF>(buf, P, s, rows, ld, tw, inverse); break;
        case 4: stage<4, DIF>(buf, P, s, rows, ld, tw, inverse); break;
        case 2: stage<2, DIF>(buf, P, s, rows, ld, tw, inverse); break;
        case 3: stage<3, DIF>(buf, P, s, rows, ld, tw, inverse); break;
        default: stage<5, DIF>(buf, P, s, rows, ld, tw, inverse); break;
    }
}

// Digit-reversed input -> natural-order transform.
__device__ void dit(cplx* buf, const FftPlan& P, int rows, int ld, const cplx* tw, bool inverse) {
    for (int s = 0; s < P.ns; ++s) {
        run_stage<false>(buf, P, s, rows, ld, tw, inverse);
        __syncthreads();
    }
}

// Natural-order input -> digit-reversed transform (the transpose of dit).
__device__ void dif(cplx* buf, const FftPlan& P, int rows, int ld, const cplx* tw, bool inverse) {
    for (int s = P.ns - 1; s >= 0; --s) {
        run_stage<true>(buf, P, s, rows, ld, tw, inverse);
        __syncthreads();
    }
}

enum RowMode { kFwdPack = 0, kFwd = 1, kInv = 2, kInvOut = 3 };

// One workgroup per row of length P.n (<= MAXN), transformed in LDS.
// kFwdPack: row of Z = M + iK from the counts and the kernel, forward, natural
//           order out. kFwd: complex row, forward. kInv: complex row, inverse,
//           natural order out. kInvOut: inverse, Re * scale to a double row.
// bal[0] = 2^e multiplies K on the way in, bal[1] = 2^-e undoes it on the way out.
template <int MAXN, int THREADS, int MODE>
__global__ void __launch_bounds__(THREADS)
row_fft_kernel(const int32_t* __restrict__ counts, const double* __restrict__ kern, cplx* z,
               double* __restrict__ out, FftPlan P, const cplx* __restrict__ tw, double scale,
               const double* __restrict__ bal) {
    __shared__ cplx buf[MAXN];
    const int n = P.n;
    const int64_t off = (int64_t)blockIdx.x * n;
    if (MODE == kFwdPack || MODE == kFwd) {
        const double sk = MODE == kFwdPack ? bal[0] : 1.0;
        for (int i = threadIdx.x; i < n; i += THREADS) {
            const int p = digit_pos(i, P);
            if (MODE == kFwdPack) buf[swz(p)] = cplx{(double)counts[off + i], kern[off + i] * sk};
            else buf[swz(p)] = z[off + i];
        }
        __syncthreads();
        dit(buf, P, 1, MAXN, tw, false);
        for (int i = threadIdx.x; i < n; i += THREADS) z[off + i] = buf[swz(i)];
    } else {
        for (int i = threadIdx.x; i < n; i += THREADS) buf[swz(i)] = z[off + i];
        __syncthreads();
        dif(buf, P, 1, MAXN, tw, true);
        const double su = MODE == kInvOut ? bal[1] : 1.0;
        for (int i = threadIdx.x; i < n; i += THREADS) {
            const cplx v = buf[swz(digit_pos(i, P))];
            if (MODE == kInvOut) out[off + i] = (v.x * scale) * su;
            else z[off + i] = v;
        }
    }
}

// Balance of the two-for-one transform. Recovering F(K) from Z = M + iK
// subtracts terms of the size of F(M), so K's spectrum would carry rounding
// errors of M's magnitude; packing Z = M + i 2^e K with 2^e close to
// ||M||_2 / ||K||_2 makes both spectra equally precise, and the power of two
// is undone exactly at the end. The norms are reduced in a fixed order
// (kNormBlocks partial sums, then one workgroup), so the result is reproducible.
constexpr int kNormBlocks = 1024;

__global__ void __launch_bounds__(256) norms_kernel(const int32_t* __restrict__ m,
                                                    const double* __restrict__ k, int64_t n,
                                                    double* __restrict__ part) {
    __shared__ double sm[256], sk[256];
    double am = 0.0, ak = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)kNormBlocks * 256) {
        const double a = (double)m[i], b = k[i];
        am += a * a;
        ak += b * b;
    }
    sm[threadIdx.x] = am;
    sk[threadIdx.x] = ak;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sm[threadIdx.x] += sm[threadIdx.x + w];
            sk[threadIdx.x] += sk[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sm[0];
        part[2 * blockIdx.x + 1] = sk[0];
    }
}

__global__ void __launch_bounds__(256) balance_kernel(const double* __restrict__ part,
                                                      double* __restrict__ bal) {
    __shared__ double sm[256], sk[256];
    double am = 0.0, ak = 0.0;
    for (int b = threadIdx.x; b < kNormBlocks; b += 256) {
        am += part[2 * b];
        ak += part[2 * b + 1];
    }
    sm[threadIdx.x] = am;
    sk[threadIdx.x] = ak;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sm[threadIdx.x] += sm[threadIdx.x + w];
            sk[threadIdx.x] += sk[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int e = 0;
        if (sm[0] > 0.0 && sk[0] > 0.0 && isfinite(sm[0]) && isfinite(sk[0])) {
            e = (int)rint(0.5 * (log2(sm[0]) - log2(sk[0])));
            e = e < -900 ? -900 : (e > 900 ? 900 : e);
        }
        bal[0] = ldexp(1.0, e);
        // a kernel of zeros convolves to zeros: the factor on the way out is
        // 0, not the rounding noise that F(M) leaves in the recovered F(K)
        bal[1] = sk[0] == 0.0 ? 0.0 : ldexp(1.0, -e);
    }
}

// F(M)(u) F(K)(u) from Z-hat(u) and Z-hat(-u) of Z = M + iK.
__device__ __forceinline__ cplx spectrum_product(cplx zu, cplx zm) {
    const cplx fm = cplx{0.5 * (zu.x + zm.x), 0.5 * (zu.y - zm.y)};   // (zu + conj zm) / 2
    const cplx dk = cplx{zu.x - zm.x, zu.y + zm.y};                    // zu - conj zm
    const cplx fk = cplx{0.5 * dk.y, -0.5 * dk.x};                     // dk / 2i
    return cmul(fm, fk);
}

// Second axis, product and first inverse axis in one pass. t holds p1 rows of
// length n2 = P.n (entry (u1, x2) after the first forward axis); workgroup u1
// takes rows u1 and (p1 - u1) mod p1, whose spectra pair up under u -> -u:
// forward DIT both, form the product of the two real signals' spectra, inverse
// DIF both, store natural order.
template <int MAXN, int THREADS>
__global__ void __launch_bounds__(THREADS)
pair_kernel(cplx* __restrict__ t, int p1, FftPlan P, const cplx* __restrict__ tw) {
    __shared__ cplx buf[2 * MAXN];
    const int n = P.n;
    const int ua = blockIdx.x, ub = (p1 - ua) % p1;
    const bool self = ua == ub;
    const int rows = self ? 1 : 2;
    cplx* A = buf;
    cplx* B = buf + MAXN;
    for (int i = threadIdx.x; i < rows * n; i += THREADS) {
        const int r = i >= n, k = i - r * n;
        buf[r * MAXN + swz(digit_pos(k, P))] = t[(int64_t)(r ? ub : ua) * n + k];
    }
    __syncthreads();
    dit(buf, P, rows, MAXN, tw, false);
    for (int u = threadIdx.x; u < n; u += THREADS) {
        const int m = (n - u) % n;
        const int su = swz(u), sm = swz(m);
        if (self) {
            if (m < u) continue;
            const cplx pr = spectrum_product(A[su], A[sm]);
            A[su] = pr;
            if (m != u) A[sm] = conj(pr);
        } else {
            const cplx pr = spectrum_product(A[su], B[sm]);
            A[su] = pr;
            B[sm] = conj(pr);
        }
    }
    __syncthreads();
    dif(buf, P, rows, MAXN, tw, true);
    for (int i = threadIdx.x; i < rows * n; i += THREADS) {
        const int r = i >= n, k = i - r * n;
        t[(int64_t)(r ? ub : ua) * n + k] = buf[r * MAXN + swz(digit_pos(k, P))];
    }
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

// Product on whole planes (used when a row pair does not fit LDS): t in the
// transposed layout (p1 rows of length n2), pairs (u, -u) by one thread.
__global__ void product_kernel(cplx* __restrict__ t, int n1, int n2) {
    const int64_t total = (int64_t)n1 * n2;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int u1 = (int)(i / n2), u2 = (int)(i % n2);
        const int64_t p = (int64_t)((n1 - u1) % n1) * n2 + (n2 - u2) % n2;
        if (p < i) continue;
        const cplx prod = spectrum_product(t[i], t[p]);
        t[i] = prod;
        if (p != i) t[p] = conj(prod);
    }
}

// ----------------------------------------------------------------------------
// power-of-two sides (256 .. 8192): three passes, register-resident FFTs
// ----------------------------------------------------------------------------
//
// Both M and K are real, so each is taken through real transforms whose
// half spectra (u1 in [0, H), H = p1 / 2 + 1) are all that the product needs:
//   A. rows: one complex FFT of two rows of M (M_j + i M_j+1) and one of two
//      rows of K, unpacked into the half spectra of the four rows and stored
//      in 128-byte chunks of eight rows per frequency (one cache line), one
//      plane for M^ and one for K^, a[x2 / 8][u1] = {M^(x2 .. x2 + 7, u1)};
//      a workgroup writes 32 bytes of each chunk, and the four row pairs of a
//      chunk are consecutive workgroups on one XCD, so lines fill in its L2;
//   B. one column u1 per workgroup: forward FFTs of both columns along x2,
//      their product, the inverse FFT along x2, stored in 64-byte chunks of
//      four rows, g[x2 / 4][u1] = {g(x2 .. x2 + 3, u1)};
//   C. four rows per workgroup: the inverse FFTs of rows x2 (two rows per
//      complex FFT, g(x2) + i g(x2 + 1), extended to u1 >= H by Hermitian
//      symmetry), whose real and imaginary parts are rows x2 and x2 + 1 of
//      C, times 1 / (p1 p2 n_avg).
// Each pass reads and writes HBM once. The axis changes go through the chunk
// layouts: pass B reads pass A's chunks eight lanes to a cache line and
// writes its column four lanes to a chunk (a chunk's neighbour in the same
// cache line belongs to the next column, the next workgroup on the same XCD);
// pass C loads whole chunks at consecutive addresses. About 68 bytes
// per pixel in all, against 20 of input and output. Rows of the same
// magnitude share a transform, so no balancing factor is needed.
//
// The FFTs are Stockham transforms with T threads of E = N / T points each:
// thread t holds the elements t + T m (m < E) between stages, reads them
// straight from global memory for the first stage and keeps the last stage's
// outputs, which are again t + T m; the stages in between exchange through an
// LDS row padded by one slot in 16. Stage s (radix R, NS = product of the
// earlier radices) turns butterfly j = t + T b (b < E / R) of inputs
// x[j + q N / R] into y[(j / NS) NS R + j % NS + q NS], after the twiddles
// w^q, w = exp(-+2 pi i (j % NS) / (NS R)) read from a table of one entry per
// j % NS and stage (p2_twiddle_kernel), its powers formed in registers.

// E = 8 points per thread (4 for N = 256): radix-8 stages, the last one of
// radix 2 or 4 where N is not a power of 8. N = 10000 (the high-resolution
// GERLUMPH maps): 1000 threads of 10 points, four radix-10 stages.
template <int N> constexpr int p2_threads() { return N == 256 ? 64 : (N == 10000 ? 1000 : N / 8); }
template <int N> constexpr int p2_stages() {
    return N == 512 ? 3 : (N == 8192 ? 5 : 4);
}
template <int N, int S> constexpr int p2_radix() {
    return N == 256 ? 4
         : N == 1024 ? (S < 3 ? 8 : 2)
         : N == 2048 ? (S < 3 ? 8 : 4)
         : N == 8192 ? (S < 4 ? 8 : 2)
         : N == 10000 ? 10
         : 8;    // 512, 4096
}
// LDS row padding: one slot in 16, one in 64 for N = 10000 (so that the row
// stays within the 160 KiB a workgroup may use).
template <int N> __device__ __forceinline__ int p2_pad(int e) { return N == 10000 ? e + (e >> 6) : e + (e >> 4); }
template <int N> constexpr int p2_lds() { return N == 10000 ? N + N / 64 + 1 : N + N / 16; }
// NS of stage S (the product of the radices before it) and the offset of its
// entries in the base-twiddle table: stage S holds exp(-2 pi i k / (NS R))
// for k < NS at p2_tw_offset<N, S>() + k.
template <int N, int S> constexpr int p2_ns() { return S == 0 ? 1 : p2_ns<N, (S > 0 ? S - 1 : 0)>() * p2_radix<N, (S > 0 ? S - 1 : 0)>(); }
template <int N, int S> constexpr int p2_tw_offset() {
    return S == 0 ? 0 : p2_tw_offset<N, (S > 0 ? S - 1 : 0)>() + p2_ns<N, (S > 0 ? S - 1 : 0)>();
}

// w^1 .. w^(R-1) from w by products (at most three roundings deep, so within a
// few units of FP64 rounding of the exact roots).
template <int R>
__device__ __forceinline__ void twiddle_powers(cplx w, cplx (&p)[R]) {
    p[1] = w;
    if constexpr (R > 2) p[2] = cmul(w, w);
    if constexpr (R > 3) p[3] = cmul(p[2], w);
    if constexpr (R > 4) { p[4] = cmul(p[2], p[2]); p[5] = cmul(p[4], w); p[6] = cmul(p[3], p[3]);
                           p[7] = cmul(p[6], w); }
    if constexpr (R > 8) { p[8] = cmul(p[4], p[4]); p[9] = cmul(p[5], p[4]); }
}

// Base twiddles of a power-of-two plan: entry e of stage s (offset off_s,
// off_0 = 0, off_s+1 = off_s + L[s]) is exp(-2 pi i k / L[s+1]), k = e - off_s.
__global__ void p2_twiddle_kernel(cplx* __restrict__ tw, FftPlan P) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    int off = 0, s = 0;
    while (s < P.ns && e >= off + P.L[s]) { off += P.L[s]; ++s; }
    if (s >= P.ns) return;
    double sn, cs;
    sincospi(2.0 * (double)(e - off) / (double)P.L[s + 1], &sn, &cs);
    tw[e] = cplx{cs, -sn};
}


// kz[0 .. n) = 0: no pair of K^ rows is known to hold zeros.
__global__ void p2_clear_kernel(uint8_t* __restrict__ kz, int n) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) kz[e] = 0;
}

// SPLIT: the stages exchange real and imaginary parts one after the other
// through an LDS row of doubles (half the LDS of a complex row, for one
// butterfly per thread and stage).
template <int N, int S, int NS, int V, int T = p2_threads<N>(), bool SPLIT = false>
__device__ __forceinline__ void p2_fft(cplx (&a)[V][N / T], cplx* __restrict__ lds,
                                       const cplx* __restrict__ tw, bool inverse) {
    constexpr int E = N / T, R = p2_radix<N, S>(), B = E / R;
    constexpr bool kLast = NS * R == N;
    static_assert(!SPLIT || (B == 1 && V == 1), "the split exchange takes one butterfly per thread");
    const double sg = inverse ? 1.0 : -1.0;
    const int t = threadIdx.x;
#pragma unroll
    for (int v = 0; v < V; ++v) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int j = t + T * b;
            const int k = (int)((unsigned)j % (unsigned)NS);
            cplx x[R];
#pragma unroll
            for (int q = 0; q < R; ++q) x[q] = a[v][b + q * B];
            if constexpr (NS > 1) {
                cplx w = tw[p2_tw_offset<N, S>() + k];
                if (inverse) w.y = -w.y;
                cplx wp[R];
                twiddle_powers<R>(w, wp);
#pragma unroll
                for (int q = 1; q < R; ++q) x[q] = cmul(x[q], wp[q]);
            }
            small_dft<R>(x, sg);
            if constexpr (kLast) {
#pragma unroll
                for (int q = 0; q < R; ++q) a[v][b + q * B] = x[q];
            } else if constexpr (SPLIT) {
                double* __restrict__ ld = reinterpret_cast<double*>(lds);
                const int base = (j / NS) * NS * R + k;
#pragma unroll
                for (int q = 0; q < R; ++q) ld[p2_pad<N>(base + q * NS)] = x[q].x;
                __syncthreads();
#pragma unroll
                for (int m = 0; m < E; ++m) a[v][m].x = ld[p2_pad<N>(t + T * m)];
                __syncthreads();
#pragma unroll
                for (int q = 0; q < R; ++q) ld[p2_pad<N>(base + q * NS)] = x[q].y;
                __syncthreads();
#pragma unroll
                for (int m = 0; m < E; ++m) a[v][m].y = ld[p2_pad<N>(t + T * m)];
                __syncthreads();
            } else {
                const int base = (j / NS) * NS * R + k;
#pragma unroll
                for (int q = 0; q < R; ++q) lds[p2_pad<N>(base + q * NS)] = x[q];
            }
        }
        if constexpr (!kLast && !SPLIT) {
            __syncthreads();
#pragma unroll
            for (int m = 0; m < E; ++m) a[v][m] = lds[p2_pad<N>(t + T * m)];
            __syncthreads();
        }
    }
    if constexpr (!kLast) p2_fft<N, S + 1, NS * R, V, T, SPLIT>(a, lds, tw, inverse);
}

// Bijective remap of a block id: blocks dispatched to the same XCD (block b
// runs on XCD b % 8) take consecutive rows, so pieces of one cache line meet
// in one L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int x = b % 8, idx = b / 8, per = nb / 8, rem = nb % 8;
    return x < rem ? x * (per + 1) + idx : rem * (per + 1) + (x - rem) * per + idx;
}

// Pass A. Block = rows j0, j0 + 1 of the p2 x N maps M and K; the M pair and
// the K pair are transformed one after the other (fewer live registers: two
// workgroups fit a CU).
// PARTS: bit 0 transforms the map's row pairs, bit 1 the kernel's (a batch of
// kernels against one map transforms the map once).
template <int N, int PARTS = 3>
__global__ void __launch_bounds__(p2_threads<N>())
__attribute__((amdgpu_waves_per_eu(N >= 2048 && N <= 4096 ? 4 : 1)))
p2_rows_fwd_kernel(const int32_t* __restrict__ M, const double* __restrict__ K, int p2,
                   cplx* __restrict__ A, const cplx* __restrict__ tw, uint8_t* __restrict__ kz,
                   int32_t* __restrict__ kseg, cplx* __restrict__ kzero) {
    constexpr int T = p2_threads<N>(), E = N / T;
    __shared__ cplx lds[p2_lds<N>()];
    __shared__ int any_nz;     // the kernel's row pair holds a nonzero value
    const int t = threadIdx.x;
    const int j0 = 2 * xcd_block(blockIdx.x, gridDim.x);
    if (t == 0) any_nz = 0;    // ordered before its use by the M pair's barriers
    if constexpr (PARTS == 2) __syncthreads();   // ... or by this one
#pragma unroll
    for (int v = 0; v < 2; ++v) {
        if (!((PARTS >> v) & 1)) continue;
        cplx a[1][E];
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int i = t + T * m;
            // streamed once: non-temporal, so they do not push the half
            // spectra's partly written lines out of L2
            if (v == 0)
                a[0][m] = cplx{(double)__builtin_nontemporal_load(&M[(int64_t)j0 * N + i]),
                               (double)__builtin_nontemporal_load(&M[(int64_t)(j0 + 1) * N + i])};
            else
                a[0][m] = cplx{__builtin_nontemporal_load(&K[(int64_t)j0 * N + i]),
                               __builtin_nontemporal_load(&K[(int64_t)(j0 + 1) * N + i])};
        }
        // A source profile is zero beyond its radius, so most row pairs of a
        // kernel are zeros, whose half spectra are zeros: those are stored
        // without a transform, and not stored at all when kz says that this
        // pair's rows of K^ already hold zeros from the previous call with the
        // same sides (the decision is the workgroup's, taken on the values it
        // has loaded; a dense kernel costs one more barrier).
        bool zero_pair = false, skip = false;
        if (v == 1) {
            bool nz = false;
#pragma unroll
            for (int m = 0; m < E; ++m) nz = nz || a[0][m].x != 0.0 || a[0][m].y != 0.0;
            if (nz) any_nz = 1;
            const bool was_zero = kz[j0 >> 1] != 0;   // read by all before thread 0 rewrites it
            __syncthreads();
            zero_pair = any_nz == 0;
            skip = zero_pair && was_zero;
            if (t == 0 && zero_pair != was_zero) kz[j0 >> 1] = zero_pair ? 1 : 0;
            // a pair that is not all zeros marks its 64-row segment: pass B
            // reads K^ only in marked segments, and pass C clears the marks
            if (t == 0 && !zero_pair) kseg[j0 >> 6] = 1;
            if (t == 0 && blockIdx.x == 0) *kzero = cplx{0.0, 0.0};
        }
        if (!zero_pair) {
            p2_fft<N, 0, 1, 1>(a, lds, tw, false);
            // unpack: X^(u) = (Z(u) + conj Z(-u)) / 2, Y^(u) = (Z(u) - conj Z(-u)) / 2i,
            // stored at once (the M^ and K^ pieces of a chunk meet in L2)
#pragma unroll
            for (int m = 0; m < E; ++m) lds[p2_pad<N>(t + T * m)] = a[0][m];
            __syncthreads();
        }
#pragma unroll
        for (int m = 0; m <= E / 2; ++m) {
            if (skip || (m == E / 2 && t != 0)) continue;     // u = N / 2 belongs to thread 0
            const int u = t + T * m;
            cplx* __restrict__ o = A + (int64_t)v * p2 * (N / 2 + 1) +
                                   ((int64_t)(j0 / 8) * (N / 2 + 1) + u) * 8 + (j0 & 7);
            if (zero_pair) {
                o[0] = cplx{0.0, 0.0};
                o[1] = cplx{0.0, 0.0};
            } else {
                const cplx zu = a[0][m];
                const cplx zm = lds[p2_pad<N>(u == 0 ? 0 : N - u)];
                o[0] = cplx{0.5 * (zu.x + zm.x), 0.5 * (zu.y - zm.y)};
                o[1] = cplx{0.5 * (zu.y + zm.y), 0.5 * (zm.x - zu.x)};
            }
        }
        __syncthreads();
        // keep the K rows' loads after the M pair's stores
        __builtin_amdgcn_sched_barrier(0);
    }
}

// A complex value read once by this workgroup (its whole cache line is read
// by the same wave): non-temporal, so it does not hold L2 lines that
// partly written outputs still need.
__device__ __forceinline__ cplx nt_load(const cplx* p) {
    return cplx{__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y)};
}

// Pass B. Block = column u1 of the half spectra (p2 = N points along x2);
// the two forward transforms run one after the other (fewer live registers:
// two workgroups fit a CU).
template <int N>
__global__ void __launch_bounds__(p2_threads<N>())
__attribute__((amdgpu_waves_per_eu(N >= 2048 && N <= 4096 ? 4 : 1)))
p2_cols_kernel(const cplx* __restrict__ A, int H, cplx* __restrict__ G, const cplx* __restrict__ tw,
               const int32_t* __restrict__ kseg, const cplx* __restrict__ kzero) {
    constexpr int T = p2_threads<N>(), E = N / T;
    // 10000-point columns: the transforms exchange through a row of doubles,
    // and the real parts of M^'s transform wait in the other half of LDS
    // while K^'s is formed, so that the two do not share the 128 registers
    // of a lane (they spilled 236 bytes per lane)
    constexpr bool kSplit = N == 10000;
    constexpr int kLdsCplx = kSplit ? (p2_lds<N>() + N + 1) / 2 : p2_lds<N>();
    __shared__ cplx lds[kLdsCplx];
    double* __restrict__ park = reinterpret_cast<double*>(lds) + p2_lds<N>();
    const int t = threadIdx.x;
    const int u1 = xcd_block(blockIdx.x, gridDim.x);
    // chunk (x2 / 8, u1) of the M^ plane, then of the K^ plane, row x2 % 8
    const cplx* __restrict__ colm = A + (int64_t)u1 * 8;
    const cplx* __restrict__ colk = colm + (int64_t)N * H;
    cplx a[1][E], b[1][E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int i = t + T * m;
        a[0][m] = nt_load(&colm[(int64_t)(i >> 3) * H * 8 + (i & 7)]);
    }
    p2_fft<N, 0, 1, 1, T, kSplit>(a, lds, tw, false);
    if constexpr (kSplit) {
#pragma unroll
        for (int m = 0; m < E; ++m) park[t + T * m] = a[0][m].x;   // read back by this thread
    }
    // keep K^'s loads after M^'s transform: hoisted, they would hold registers
    // through it
    __builtin_amdgcn_sched_barrier(0);
    // Rows of K^ in 64-row segments that pass A did not mark are zeros: the
    // wave reads them from the one zero that pass A stores (a cached line,
    // no HBM traffic). The wave's 64 rows lie in at most two segments, so
    // the test is wave-uniform; the loads stay unconditional, with base and
    // offset switched by a select and a mask (loads under a branch here gave
    // wrong results on 8192-point columns).
    const int w0 = __builtin_amdgcn_readfirstlane(t & ~63);
    // the thread index through an empty asm: the offsets below are formed
    // here, not shared with those of M^'s loads and held in registers through
    // its transform (which spilled them)
    int tk = t;
    asm volatile("" : "+v"(tk));
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int i = tk + T * m;
        const int r0 = w0 + T * m;
        const int32_t need = kseg[r0 >> 6] | kseg[(r0 + 63) >> 6];
        const int64_t mask = need != 0 ? -1 : 0;
        const cplx* base = need != 0 ? colk : kzero;
        const int64_t off = ((int64_t)(i >> 3) * H * 8 + (i & 7)) & mask;
        b[0][m] = nt_load(base + off);
    }
    p2_fft<N, 0, 1, 1, T, kSplit>(b, lds, tw, false);
    if constexpr (kSplit) {
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int m = 0; m < E; ++m) a[0][m].x = park[t + T * m];
    }
#pragma unroll
    for (int m = 0; m < E; ++m) a[0][m] = cmul(a[0][m], b[0][m]);
    p2_fft<N, 0, 1, 1, T, kSplit>(a, lds, tw, true);
    // chunk (x2 / 4, u1) holds rows x2 .. x2 + 3 (four consecutive lanes);
    // the offsets are formed here (the index through an empty asm, as above)
    int tg = t;
    asm volatile("" : "+v"(tg));
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int i = tg + T * m;
        G[((int64_t)(i >> 2) * H + u1) * 4 + (i & 3)] = a[0][m];
    }
}

// Output rows per workgroup of pass C: four (two complex transforms), two for
// N = 10000, whose transforms alone fill the 128 registers of a lane.
template <int N> constexpr int p2_inv_rows() { return N == 10000 ? 2 : 4; }

// Pass C. Block = rows j0 .. j0 + RW - 1 of the output (p1 = N points along x1).
template <int N>
__global__ void __launch_bounds__(p2_threads<N>())
__attribute__((amdgpu_waves_per_eu(N >= 2048 && N <= 4096 ? 4 : 1)))
p2_rows_inv_kernel(const cplx* __restrict__ G, int p2, double scale, double* __restrict__ out,
                   const cplx* __restrict__ tw, int32_t* __restrict__ kseg) {
    constexpr int T = p2_threads<N>(), E = N / T, H = N / 2 + 1, RW = p2_inv_rows<N>(), V = RW / 2;
    __shared__ cplx lds[p2_lds<N>()];
    const int t = threadIdx.x;
    // pass B has read the segment marks: cleared for the next call's pass A
    if (blockIdx.x == 0)
        for (int e = t; e < p2 / 64 + 2; e += T) kseg[e] = 0;
    const int j0 = RW * xcd_block(blockIdx.x, gridDim.x);
    cplx a[V][E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int u = t + T * m;
        const bool mirror = u >= H;
        const int src = mirror ? N - u : u;
        // chunk (j0 / 4, src) holds rows 4 (j0 / 4) .. + 3
        const cplx* __restrict__ c = G + ((int64_t)(j0 / 4) * H + src) * 4 + (j0 & 3);
        // g(x2) + i g(x2 + 1), or its value at -u: conj g(x2) + i conj g(x2 + 1)
        if constexpr (V == 2) {
            const cplx c0 = c[0], c1 = c[1], c2 = c[2], c3 = c[3];
            if (!mirror) {
                a[0][m] = cplx{c0.x - c1.y, c0.y + c1.x};
                a[V - 1][m] = cplx{c2.x - c3.y, c2.y + c3.x};
            } else {
                a[0][m] = cplx{c0.x + c1.y, c1.x - c0.y};
                a[V - 1][m] = cplx{c2.x + c3.y, c3.x - c2.y};
            }
        } else {
            const cplx c0 = c[0], c1 = c[1];
            a[0][m] = mirror ? cplx{c0.x + c1.y, c1.x - c0.y} : cplx{c0.x - c1.y, c0.y + c1.x};
        }
    }
    p2_fft<N, 0, 1, V, T>(a, lds, tw, true);
    double* __restrict__ o = out + (int64_t)j0 * N;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int i = t + T * m;
        // written once and not read back here: non-temporal
        __builtin_nontemporal_store(a[0][m].x * scale, &o[i]);
        __builtin_nontemporal_store(a[0][m].y * scale, &o[N + i]);
        if constexpr (V == 2) {
            __builtin_nontemporal_store(a[V - 1][m].x * scale, &o[2 * N + i]);
            __builtin_nontemporal_store(a[V - 1][m].y * scale, &o[3 * N + i]);
        }
    }
}

// Sides of the three-pass path: powers of two from 256 to 8192, and 10000.
bool pow2_side(int n) {
    return n == 256 || n == 512 || n == 1024 || n == 2048 || n == 4096 || n == 8192 || n == 10000;
}

// The stage radices of a power-of-two side as an FftPlan (for the base
// twiddle table: L[s] = NS of stage s).
template <int N>
FftPlan p2_plan() {
    FftPlan P{};
    P.n = N;
    P.ns = p2_stages<N>();
    const int r[5] = {p2_radix<N, 0>(), p2_radix<N, 1>(), p2_radix<N, 2>(), p2_radix<N, 3>(),
                      p2_radix<N, 4>()};
    P.L[0] = 1;
    for (int s = 0; s < P.ns; ++s) {
        P.r[s] = r[s];
        P.L[s + 1] = P.L[s] * r[s];
        P.div[s] = 0;
    }
    return P;
}

FftPlan p2_plan_of(int n) {
    switch (n) {
        case 256: return p2_plan<256>();
        case 512: return p2_plan<512>();
        case 1024: return p2_plan<1024>();
        case 2048: return p2_plan<2048>();
        case 4096: return p2_plan<4096>();
        case 8192: return p2_plan<8192>();
        default: return p2_plan<10000>();
    }
}

template <int N>
hipError_t p2_rows_fwd(int parts, const int32_t* M, const double* K, int p2, cplx* A, const cplx* tw, uint8_t* kz,
                       int32_t* kseg, cplx* kzero, hipStream_t s) {
    auto k = parts == 1 ? p2_rows_fwd_kernel<N, 1> : (parts == 2 ? p2_rows_fwd_kernel<N, 2> : p2_rows_fwd_kernel<N, 3>);
    hipLaunchKernelGGL(k, dim3(p2 / 2), dim3(p2_threads<N>()), 0, s, M, K, p2, A, tw, kz, kseg, kzero);
    return hipGetLastError();
}
template <int N>
hipError_t p2_cols(const cplx* A, cplx* G, int H, const cplx* tw, const int32_t* kseg, const cplx* kzero,
                   hipStream_t s) {
    hipLaunchKernelGGL(p2_cols_kernel<N>, dim3(H), dim3(p2_threads<N>()), 0, s, A, H, G, tw, kseg, kzero);
    return hipGetLastError();
}
template <int N>
hipError_t p2_rows_inv(const cplx* G, int p2, double scale, double* out, const cplx* tw, int32_t* kseg,
                       hipStream_t s) {
    hipLaunchKernelGGL(p2_rows_inv_kernel<N>, dim3(p2 / p2_inv_rows<N>()), dim3(p2_threads<N>()), 0, s, G, p2, scale,
                       out, tw, kseg);
    return hipGetLastError();
}

hipError_t p2_rows_fwd_any(int n, int parts, const int32_t* M, const double* K, int p2, cplx* A, const cplx* tw,
                           uint8_t* kz, int32_t* kseg, cplx* kzero, hipStream_t s) {
#define RL_CALL(N) p2_rows_fwd<N>(parts, M, K, p2, A, tw, kz, kseg, kzero, s)
    switch (n) {
        case 256: return RL_CALL(256);
        case 512: return RL_CALL(512);
        case 1024: return RL_CALL(1024);
        case 2048: return RL_CALL(2048);
        case 4096: return RL_CALL(4096);
        case 8192: return RL_CALL(8192);
        default: return RL_CALL(10000);
    }
#undef RL_CALL
}
hipError_t p2_cols_any(int n, const cplx* A, cplx* G, int H, const cplx* tw, const int32_t* kseg,
                       const cplx* kzero, hipStream_t s) {
#define RL_CALL(N) p2_cols<N>(A, G, H, tw, kseg, kzero, s)
    switch (n) {
        case 256: return RL_CALL(256);
        case 512: return RL_CALL(512);
        case 1024: return RL_CALL(1024);
        case 2048: return RL_CALL(2048);
        case 4096: return RL_CALL(4096);
        case 8192: return RL_CALL(8192);
        default: return RL_CALL(10000);
    }
#undef RL_CALL
}
hipError_t p2_rows_inv_any(int n, const cplx* G, int p2, double scale, double* out, const cplx* tw,
                           int32_t* kseg, hipStream_t s) {
#define RL_CALL(N) p2_rows_inv<N>(G, p2, scale, out, tw, kseg, s)
    switch (n) {
        case 256: return RL_CALL(256);
        case 512: return RL_CALL(512);
        case 1024: return RL_CALL(1024);
        case 2048: return RL_CALL(2048);
        case 4096: return RL_CALL(4096);
        case 8192: return RL_CALL(8192);
        default: return RL_CALL(10000);
    }
#undef RL_CALL
}

size_t p2_scratch_bytes(int p1, int p2) {
    const size_t h = (size_t)(p1 / 2 + 1) * p2;
    // planes A (two) and G, the twiddles, one zero, the pair flags (16-byte
    // padded) and the segment marks
    return h * 3 * sizeof(cplx) + (size_t)(p1 + p2 + 1) * sizeof(cplx) + (size_t)(p2 + 15) / 16 * 16 +
           (size_t)(p2 / 64 + 2) * sizeof(int32_t) + 256;
}

// A map against n kernels: the map's row transforms once (pass A, map part),
// then per kernel pass A's kernel part, pass B and pass C; with n = 1 pass A
// does both parts in one launch.
hipError_t p2_convolve(const int32_t* counts, const double* const* kernels, int n, int p1, int p2,
                       double n_avg, double* const* outs, void* scratch, bool twiddles_ready, hipStream_t s) {
    const int H = p1 / 2 + 1;
    cplx* A = static_cast<cplx*>(scratch);                 // {M^, K^} x p2 / 8 x H x {eight rows}
    cplx* G = A + (size_t)H * p2 * 2;                      // p2 / 4 x H x {4 rows}
    cplx* tw1 = G + (size_t)H * p2;                        // stage twiddles along x1
    cplx* tw2 = tw1 + p1;                                  // ... along x2
    cplx* kzero = tw2 + p2;                                // one zero for pass B
    // p2 / 2 flags: the pair's rows of K^ hold zeros (kept with the twiddles:
    // valid while the sides and the scratch buffer stay the same)
    uint8_t* kz = reinterpret_cast<uint8_t*>(kzero + 1);
    // p2 / 64 + 2 segment marks (room for pass B's last wave to look one
    // segment past the end)
    int32_t* kseg = reinterpret_cast<int32_t*>(kz + ((p2 + 15) / 16) * 16);
    if (!twiddles_ready) {
        const FftPlan P1 = p2_plan_of(p1), P2 = p2_plan_of(p2);
        hipLaunchKernelGGL(p2_twiddle_kernel, dim3((p1 + 255) / 256), dim3(256), 0, s, tw1, P1);
        hipLaunchKernelGGL(p2_twiddle_kernel, dim3((p2 + 255) / 256), dim3(256), 0, s, tw2, P2);
        hipLaunchKernelGGL(p2_clear_kernel, dim3((p2 / 2 + 255) / 256), dim3(256), 0, s, kz, p2 / 2);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && n > 1) e = p2_rows_fwd_any(p1, 1, counts, nullptr, p2, A, tw1, kz, kseg, kzero, s);
    const double scale = 1.0 / ((double)p1 * (double)p2 * n_avg);
    for (int q = 0; q < n && e == hipSuccess; ++q) {
        e = p2_rows_fwd_any(p1, n > 1 ? 2 : 3, counts, kernels[q], p2, A, tw1, kz, kseg, kzero, s);
        if (e == hipSuccess) e = p2_cols_any(p2, A, G, H, tw2, kseg, kzero, s);
        if (e == hipSuccess) e = p2_rows_inv_any(p1, G, p2, scale, outs[q], tw1, kseg, s);
    }
    return e;
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

// Pixel (i, j), |i| <= h1, |j| <= h2, gets the mean brightness over an 8 x 8
// grid of sub-samples, stored compactly at q = (j + h2) (2 h1 + 1) + (i + h1).
// One wave per pixel, lane l on sub-sample (l mod 8, l / 8); the 64 values are
// summed in a fixed butterfly order.
constexpr int kSourceSub = 8;
__global__ void __launch_bounds__(256) source_samples_kernel(int shape, double radius, double hole, double pix1,
                                                             double pix2, int h1, int h2,
                                                             double* __restrict__ compact) {
    const int w = 2 * h1 + 1;
    const int64_t total = (int64_t)w * (2 * h2 + 1);
    const int lane = threadIdx.x % 64;
    const double ox = ((double)(lane % kSourceSub) + 0.5) / (double)kSourceSub - 0.5;
    const double oy = ((double)(lane / kSourceSub) + 0.5) / (double)kSourceSub - 0.5;
    const int wpb = blockDim.x / 64;
    for (int64_t q = (int64_t)blockIdx.x * wpb + threadIdx.x / 64; q < total; q += (int64_t)gridDim.x * wpb) {
        const int i = (int)(q % w) - h1, j = (int)(q / w) - h2;
        const double x = ((double)i + ox) * pix1;
        const double y = ((double)j + oy) * pix2;
        double v = brightness(shape, hypot(x, y), radius, hole);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) compact[q] = v / (double)(kSourceSub * kSourceSub);
    }
}

// One workgroup, fixed summation order (four loads in flight per thread, then
// a fixed tree): the normalisation is reproducible.
__global__ void __launch_bounds__(1024) ordered_sum_kernel(const double* __restrict__ v, int64_t n,
                                                           double* __restrict__ out) {
    __shared__ double part[1024];
    const int t = threadIdx.x;
    double s = 0.0;
    int64_t i = t;
    for (; i + 3 * 1024 < n; i += 4 * 1024) {
        const double a = v[i], b = v[i + 1024], c = v[i + 2048], d = v[i + 3072];
        s += a;
        s += b;
        s += c;
        s += d;
    }
    for (; i < n; i += 1024) s += v[i];
    part[t] = s;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if (t < h) part[t] += part[t + h];
        __syncthreads();
    }
    if (t == 0) *out = part[0];
}

// The whole p2 x p1 kernel in one pass, row jj = blockIdx.y: pixel (ii, jj)
// holds compact[(j + h2) (2 h1 + 1) + (i + h1)] / total for the offsets
// i = ii or ii - p1, j = jj or jj - p2 inside the source box, 0 elsewhere
// (2 h + 1 <= p on both axes, so no two offsets meet).
__global__ void __launch_bounds__(256) fill_source_kernel(const double* __restrict__ compact, int h1, int h2,
                                                          int p1, int p2, const double* __restrict__ total,
                                                          double* __restrict__ k) {
    const int jj = blockIdx.y;
    const int ii = blockIdx.x * blockDim.x + threadIdx.x;
    if (ii >= p1) return;
    const int j = jj <= h2 ? jj : jj - p2;
    const int i = ii <= h1 ? ii : ii - p1;
    double v = 0.0;
    if (j >= -h2 && j <= h2 && i >= -h1 && i <= h1) v = compact[(int64_t)(j + h2) * (2 * h1 + 1) + (i + h1)] / *total;
    k[(int64_t)jj * p1 + ii] = v;
}

// Tabulated profiles. Sample k of an axis with positions v lies in pixel
// floor(v[k] / pix + 1/2), taken in FP64 from the FP32 position; bins[k] holds
// that pixel + h (0 .. 2 h). The x and y axes share one launch: k < nx is x.
__global__ void __launch_bounds__(256) table_bins_kernel(const float* __restrict__ x, int nx,
                                                         const float* __restrict__ y, int ny, double pix1,
                                                         double pix2, int h1, int h2, int32_t* __restrict__ bins) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nx) bins[k] = (int)floor((double)x[k] / pix1 + 0.5) + h1;
    else if (k < nx + ny) bins[k] = (int)floor((double)y[k - nx] / pix2 + 0.5) + h2;
}

// Stable bucket order of one axis (n samples, bins 0 .. nb - 1): sample k goes
// to order[start[bin k] + number of earlier samples in its bin], start[b] =
// number of samples in bins below b, start[nb] = n. One wave per output: wave
// w < n ranks sample w, wave n + b counts start[b]; its lanes split the axis
// and a butterfly adds their counts (thousands of waves: the quadratic count
// is spread over the whole chip instead of a few workgroups).
__global__ void __launch_bounds__(256) table_order_kernel(const int32_t* __restrict__ bins, int n, int nb,
                                                          int32_t* __restrict__ order, int32_t* __restrict__ start) {
    const int lane = threadIdx.x % 64;
    const int w = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64);
    if (w > n + nb) return;     // wave-uniform
    const bool rank = w < n;
    const int bt = rank ? bins[w] : w - n;
    int cnt = 0;
    for (int k = lane; k < n; k += 64) {
        const int b = bins[k];
        cnt += rank ? ((b < bt) | ((b == bt) & (k < w))) : (b < bt);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
    if (lane == 0) {
        if (rank) order[cnt] = w;
        else start[bt] = cnt;
    }
}

// Pixel (i, j) of the compact (2 h1 + 1) x (2 h2 + 1) box sums the brightness
// of the samples it holds: one wave per pixel, item e of its rows x columns
// product (table order, rows outer) on lane e mod 64, each lane summing its
// items in order, then a fixed butterfly. Reproducible, and equal to the sum in
// table order up to rounding; a paper-sized table (1000 - 3000 points per axis)
// puts hundreds of samples in each pixel.
__global__ void __launch_bounds__(256) table_samples_kernel(const float* __restrict__ b, int nx,
                                                            const int32_t* __restrict__ ox,
                                                            const int32_t* __restrict__ sx,
                                                            const int32_t* __restrict__ oy,
                                                            const int32_t* __restrict__ sy, int h1, int h2,
                                                            double* __restrict__ compact) {
    const int w = 2 * h1 + 1;
    const int64_t total = (int64_t)w * (2 * h2 + 1);
    const int lane = threadIdx.x % 64;
    const int wpb = blockDim.x / 64;
    for (int64_t q = (int64_t)blockIdx.x * wpb + threadIdx.x / 64; q < total; q += (int64_t)gridDim.x * wpb) {
        const int i = (int)(q % w), j = (int)(q / w);
        const int a0 = sy[j], c0 = sx[i], nc = sx[i + 1] - c0;
        const int ne = (sy[j + 1] - a0) * nc;
        double s = 0.0;
        for (int e = lane; e < ne; e += 64) {
            const int a = e / nc, c = e - a * nc;
            s += (double)b[(int64_t)oy[a0 + a] * nx + ox[c0 + c]];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
        if (lane == 0) compact[q] = s;
    }
}

int grid_of(int64_t n, int cap) {
    int64_t g = (n + 255) / 256;
    return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

// LDS size classes: rows up to 1024 / 4096 / 10240 points (16 / 64 / 160 KiB),
// row pairs up to 512 / 2048 / 5120 points.
// Threads per workgroup of the row and row-pair kernels for a length n.
int row_threads(int n) { return n <= 1024 ? 256 : (n <= 4096 ? 512 : 1024); }
int pair_threads(int n) { return n <= 512 ? 256 : (n <= 2048 ? 512 : 1024); }

// Largest power-of-two radix r <= 16 with at least `threads` butterflies per
// stage over `rows` rows of length n.
int max_radix(int n, int rows, int threads) {
    int r = 16;
    while (r > 4 && (int64_t)rows * n / r < threads) r >>= 1;
    return r;
}

template <int MODE>
hipError_t rows(const int32_t* counts, const double* kern, cplx* z, double* out, int nrows,
                const FftPlan& P, const cplx* tw, double scale, const double* bal, hipStream_t s) {
    if (P.n <= 1024)
        hipLaunchKernelGGL((row_fft_kernel<1024, 256, MODE>), dim3(nrows), dim3(256), 0, s, counts, kern,
                           z, out, P, tw, scale, bal);
    else if (P.n <= 4096)
        hipLaunchKernelGGL((row_fft_kernel<4096, 512, MODE>), dim3(nrows), dim3(512), 0, s, counts, kern,
                           z, out, P, tw, scale, bal);
    else
        hipLaunchKernelGGL((row_fft_kernel<kMaxFftSide, 1024, MODE>), dim3(nrows), dim3(1024), 0, s,
                           counts, kern, z, out, P, tw, scale, bal);
    return hipGetLastError();
}

hipError_t pairs(cplx* t, int p1, const FftPlan& P, const cplx* tw, hipStream_t s) {
    const dim3 grid(p1 / 2 + 1);
    if (P.n <= 512)
        hipLaunchKernelGGL((pair_kernel<512, 256>), grid, dim3(256), 0, s, t, p1, P, tw);
    else if (P.n <= 2048)
        hipLaunchKernelGGL((pair_kernel<2048, 512>), grid, dim3(512), 0, s, t, p1, P, tw);
    else
        hipLaunchKernelGGL((pair_kernel<kMaxFftSide / 2, 1024>), grid, dim3(1024), 0, s, t, p1, P, tw);
    return hipGetLastError();
}

hipError_t transpose(const cplx* in, cplx* out, int rows, int cols, hipStream_t s) {
    hipLaunchKernelGGL(transpose_kernel, dim3((cols + 31) / 32, (rows + 31) / 32), dim3(256), 0, s, in,
                       out, rows, cols);
    return hipGetLastError();
}

}  // namespace

bool fft_side_supported(int n) {
    FftPlan P;
    return n >= 2 && n <= kMaxFftSide && make_plan(n, &P);
}

size_t convolve_scratch_bytes(int p1, int p2) {
    if (pow2_side(p1) && pow2_side(p2)) return p2_scratch_bytes(p1, p2);
    const size_t plane = (size_t)p1 * p2 * sizeof(cplx);
    return 2 * plane + (size_t)(p1 + 2 * p2) * sizeof(cplx) + (2 * kNormBlocks + 2) * sizeof(double) + 256;
}

// Other sides: five passes per kernel.
hipError_t general_convolve(const int32_t* counts, const double* kernel, int p1, int p2, double n_avg,
                            double* out, void* scratch, bool twiddles_ready, hipStream_t s) {
    // plans for the x1 rows, the x2 row pairs and (long columns) the x2 rows
    FftPlan P1, P2, P2r;
    if (p1 > kMaxFftSide || p2 > kMaxFftSide || !make_plan(p1, &P1, max_radix(p1, 1, row_threads(p1))) ||
        !make_plan(p2, &P2, max_radix(p2, 2, pair_threads(p2))) ||
        !make_plan(p2, &P2r, max_radix(p2, 1, row_threads(p2))))
        return hipErrorInvalidValue;
    const int64_t n = (int64_t)p1 * p2;
    cplx* z = static_cast<cplx*>(scratch);              // p2 x p1
    cplx* t = z + n;                                    // p1 x p2
    cplx* tw1 = t + n;                                  // stage twiddles of P1
    cplx* tw2 = tw1 + p1;                               // ... of P2 (row pairs)
    cplx* tw2r = tw2 + p2;                              // ... of P2r (rows)
    double* part = reinterpret_cast<double*>(tw2r + p2); // kNormBlocks x {|M|^2, |K|^2}
    double* bal = part + 2 * kNormBlocks;               // {2^e, 2^-e}
    if (!twiddles_ready) {
        hipLaunchKernelGGL(stage_twiddle_kernel, dim3((p1 + 255) / 256), dim3(256), 0, s, tw1, P1);
        hipLaunchKernelGGL(stage_twiddle_kernel, dim3((p2 + 255) / 256), dim3(256), 0, s, tw2, P2);
        hipLaunchKernelGGL(stage_twiddle_kernel, dim3((p2 + 255) / 256), dim3(256), 0, s, tw2r, P2r);
    }
    hipLaunchKernelGGL(norms_kernel, dim3(kNormBlocks), dim3(256), 0, s, counts, kernel, n, part);
    hipLaunchKernelGGL(balance_kernel, dim3(1), dim3(256), 0, s, part, bal);
    // forward along x1 (rows of the map), Z = M + i 2^e K packed on the way in
    hipError_t e = rows<kFwdPack>(counts, kernel, z, nullptr, p2, P1, tw1, 1.0, bal, s);
    if (e == hipSuccess) e = transpose(z, t, p2, p1, s);            // t: p1 x p2
    if (e != hipSuccess) return e;
    if (p2 <= kMaxFftSide / 2) {
        e = pairs(t, p1, P2, tw2, s);                               // x2 forward, product, x2 inverse
    } else {
        e = rows<kFwd>(nullptr, nullptr, t, nullptr, p1, P2r, tw2r, 1.0, bal, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(product_kernel, dim3(grid_of(n, 8192)), dim3(256), 0, s, t, p1, p2);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = rows<kInv>(nullptr, nullptr, t, nullptr, p1, P2r, tw2r, 1.0, bal, s);
    }
    if (e == hipSuccess) e = transpose(t, z, p1, p2, s);            // z: p2 x p1
    if (e == hipSuccess)
        e = rows<kInvOut>(nullptr, nullptr, z, out, p2, P1, tw1, 1.0 / ((double)n * n_avg), bal, s);
    return e;
}

hipError_t launch_convolve(const int32_t* counts, const double* const* kernels, int n, int p1, int p2,
                           double n_avg, double* const* outs, void* scratch, bool twiddles_ready, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (pow2_side(p1) && pow2_side(p2))
        return p2_convolve(counts, kernels, n, p1, p2, n_avg, outs, scratch, twiddles_ready, s);
    hipError_t e = hipSuccess;
    for (int q = 0; q < n && e == hipSuccess; ++q)
        e = general_convolve(counts, kernels[q], p1, p2, n_avg, outs[q], scratch, twiddles_ready || q > 0, s);
    return e;
}

size_t source_scratch_bytes(int h1, int h2) {
    return ((size_t)(2 * h1 + 1) * (2 * h2 + 1) + 2) * sizeof(double) + 256;
}

// Table scratch: total (2 doubles), compact box, then int32 bins (nx + ny),
// orders (nx + ny), starts (2 h1 + 2, 2 h2 + 2), then the FP32 table
// (x, y, b) that the caller copies in at table_data_offset.
size_t table_data_offset(int nx, int ny, int h1, int h2) {
    const size_t ints = 2 * ((size_t)nx + ny) + (2 * (size_t)h1 + 2) + (2 * (size_t)h2 + 2);
    const size_t off = ((size_t)(2 * h1 + 1) * (2 * h2 + 1) + 2) * sizeof(double) + ints * sizeof(int32_t);
    return (off + 255) & ~(size_t)255;
}

size_t table_scratch_bytes(int nx, int ny, int h1, int h2) {
    return table_data_offset(nx, ny, h1, h2) + ((size_t)nx + ny + (size_t)nx * ny) * sizeof(float) + 256;
}

hipError_t launch_table_kernel(int nx, int ny, double pix1, double pix2, int h1, int h2, int p1, int p2,
                               double* kernel, void* scratch, hipStream_t s) {
    const int64_t m = (int64_t)(2 * h1 + 1) * (2 * h2 + 1);
    double* total = static_cast<double*>(scratch);
    double* compact = total + 2;
    int32_t* bins = reinterpret_cast<int32_t*>(compact + m);
    int32_t* ox = bins + nx + ny;
    int32_t* oy = ox + nx;
    int32_t* sx = oy + ny;
    int32_t* sy = sx + 2 * h1 + 2;
    const float* x = reinterpret_cast<const float*>(static_cast<char*>(scratch) + table_data_offset(nx, ny, h1, h2));
    const float* y = x + nx;
    const float* b = y + ny;
    hipLaunchKernelGGL(table_bins_kernel, dim3((nx + ny + 255) / 256), dim3(256), 0, s, x, nx, y, ny, pix1, pix2,
                       h1, h2, bins);
    // one wave per sample and per start entry: n + nb + 1 waves, four per workgroup
    hipLaunchKernelGGL(table_order_kernel, dim3((nx + 2 * h1 + 2 + 3) / 4), dim3(256), 0, s, bins, nx, 2 * h1 + 1,
                       ox, sx);
    hipLaunchKernelGGL(table_order_kernel, dim3((ny + 2 * h2 + 2 + 3) / 4), dim3(256), 0, s, bins + nx, ny,
                       2 * h2 + 1, oy, sy);
    hipLaunchKernelGGL(table_samples_kernel, dim3((unsigned)std::min<int64_t>((m + 3) / 4, 65536)), dim3(256), 0,
                       s, b, nx, ox, sx, oy, sy, h1, h2, compact);
    hipLaunchKernelGGL(ordered_sum_kernel, dim3(1), dim3(1024), 0, s, compact, m, total);
    hipLaunchKernelGGL(fill_source_kernel, dim3((p1 + 255) / 256, p2), dim3(256), 0, s, compact, h1, h2, p1,
                       p2, total, kernel);
    return hipGetLastError();
}

hipError_t launch_source_kernel(int shape, double radius, double hole, double pix1, double pix2,
                                int h1, int h2, int p1, int p2, double* kernel, double* scratch,
                                hipStream_t s) {
    const int64_t m = (int64_t)(2 * h1 + 1) * (2 * h2 + 1);
    double* total = scratch;
    double* compact = scratch + 2;
    hipLaunchKernelGGL(source_samples_kernel, dim3((unsigned)std::min<int64_t>((m + 3) / 4, 65536)), dim3(256), 0,
                       s, shape, radius, hole, pix1, pix2, h1, h2, compact);
    hipLaunchKernelGGL(ordered_sum_kernel, dim3(1), dim3(1024), 0, s, compact, m, total);
    hipLaunchKernelGGL(fill_source_kernel, dim3((p1 + 255) / 256, p2), dim3(256), 0, s, compact, h1, h2, p1,
                       p2, total, kernel);
    return hipGetLastError();
}

}  // namespace rl
