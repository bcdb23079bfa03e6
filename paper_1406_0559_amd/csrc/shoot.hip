// HIP kernels for direct inverse ray-shooting on gfx950 (CDNA4).
//
// Method: Vernardos & Fluke 2014, Section 2.1. Each ray x of a regular grid is
// mapped to y = diag(1-gamma, 1+gamma) x - kappa_s x - sum_k m_k (x-x_k)/|x-x_k|^2
// (eq. 1) and counted in a source-plane pixel; mu = N_ij / N_avg (eq. 4).
//
// Work decomposition (MI355X-first, not the paper's CUDA design):
//   * A "cell" is a fixed 1024-ray tile of the ray grid (cx x cy rays, shape
//     chosen from the grid spacing so it is roughly square on the sky). One
//     wave of 64 lanes processes one cell, each lane holding a KX x KY block
//     of 16 rays in registers, or two cells, each on half of the lanes with
//     32 rays per lane (fewer per-lens differences per ray, more
//     registers). Rays of a lane share their x1 (per column) and x2 (per
//     row) offsets, so per lens a lane computes KX + KY differences and then
//     per ray one fma for r^2, half a v_rcp_f32 and 1.5 multiplies (two rays
//     share one reciprocal) and two fma.
//   * Lenses are staged per wave into LDS in tiles and read back as
//     broadcasts (every lane reads the same address). For the FP32 path each
//     lens is rebased to the cell centre while staging, from an FP32 hi/lo
//     split of its FP64 position, so FP32 differences carry an error of
//     ~eps32 * (cell size) instead of ~eps32 * |x|.
//   * The FP32 deflection sum is blocked: kBlock lenses are summed in plain
//     FP32, block sums are added into a (sum, compensation) pair by TwoSum.
//     The block size and the cells are constants of the grid, so the kernel
//     shape (rays per lane, lens tile, waves, binning mode, batching) never
//     changes a result bit.
//   * The final y = a x - alpha, the pixel test and the index are FP64 in the
//     same operation order as a plain sequential evaluation.
//   * Binning: either one global int32 atomic per binned ray, or an
//     LDS-privatised 64 x 64 sub-map per workgroup centred on the mean pixel
//     of its rays, flushed with one global atomic per touched pixel; rays
//     that fall outside the sub-map go straight to global memory.
//   * Block index -> cell mapping is XCD-aware: consecutive cells (adjacent
//     on the sky, hence adjacent on the source plane) go to workgroups that
//     run on the same XCD, so their atomics meet in the same L2.
#include <climits>
#include <mutex>

#include "internal.h"

namespace rl {
namespace {

// ----------------------------------------------------------------------------
// small helpers
// ----------------------------------------------------------------------------

// Rounded FP32 value of (hi + lo) - (ch + cl) from FP32 hi/lo splits, using
// Knuth's TwoSum for hi - ch so the leading cancellation is exact.
__device__ __forceinline__ float rebase(float hi, float lo, float ch, float cl) {
    const float s = hi - ch;
    const float bb = s - hi;
    const float e = (hi - (s - bb)) + ((-ch) - bb);
    return s + (e + (lo - cl));
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// Workgroup header in LDS: [0..2] sums of ix, iy and the binned count,
// [3] the batch work item, [4..7] bounding box (min x, min y, max x, max y),
// [8] escaped rays.
__device__ __forceinline__ void reset_header(int* hdr) {
    hdr[0] = 0; hdr[1] = 0; hdr[2] = 0;
    hdr[4] = INT_MAX; hdr[5] = INT_MAX; hdr[6] = -1; hdr[7] = -1;
    hdr[8] = 0;
}

// Bijective remap of a linear block id so that blocks dispatched to the same
// XCD (round-robin, block b -> XCD b % 8) receive consecutive work.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
    const int64_t x = b % 8, idx = b / 8, per = nb / 8, rem = nb % 8;
    return x < rem ? x * (per + 1) + idx : rem * (per + 1) + (x - rem) * per + idx;
}

// ----------------------------------------------------------------------------
// deflection sums
// ----------------------------------------------------------------------------

// Differences of the lane's rays to lens k: dx per column, dy and dy^2 per
// row. With masses the differences are divided by the lens mass: for
// d' = d / m and r'^2 = r^2 / m^2, d' / r'^2 = m d / r^2, so the mass costs
// nothing per ray. The staged entry holds (x_k / m, y_k / m, 1 / m), and
// d' = x (1/m) - x_k / m is one fma per column or row, as d = x - x_k is.
template <int KX, int KY, bool MASS>
struct LensTerms {
    float dx[KX], dy[KY], dy2[KY];

    __device__ __forceinline__ LensTerms(const float* __restrict__ wl, int k, const float (&ox)[KX],
                                         const float (&oy)[KY]) {
        if constexpr (MASS) {
            const float4 v = reinterpret_cast<const float4*>(wl)[k];
#pragma unroll
            for (int a = 0; a < KX; ++a) dx[a] = __builtin_fmaf(ox[a], v.z, -v.x);
#pragma unroll
            for (int b = 0; b < KY; ++b) dy[b] = __builtin_fmaf(oy[b], v.z, -v.y);
        } else {
            const float2 v = reinterpret_cast<const float2*>(wl)[k];
#pragma unroll
            for (int a = 0; a < KX; ++a) dx[a] = ox[a] - v.x;
#pragma unroll
            for (int b = 0; b < KY; ++b) dy[b] = oy[b] - v.y;
        }
#pragma unroll
        for (int b = 0; b < KY; ++b) dy2[b] = dy[b] * dy[b];
    }
};

// One lens against the lane's rays. Rays come in pairs (same column, grid rows
// 2m and 2m + 1; KY is even and cells start on even rows, so the pair is a
// property of the ray grid, not of the kernel shape). Both reciprocals of a
// pair come from one v_rcp_f32: q = 1 / (r2_a r2_b), 1 / r2_a = r2_b q,
// 1 / r2_b = r2_a q (3 multiplies replace a reciprocal, which issues at about a
// third of the plain FP32 rate). A product that underflows to zero (a ray on
// a lens) makes the pair's block sums non-finite; deflect_f32 then redoes that
// pair's block with one reciprocal per ray (lens_step_f32_single).
// Phase-ordered in groups of up to 16 rays: all r^2, then all reciprocals,
// then all accumulations, so no v_rcp_f32 result is consumed right after it
// issues.
template <int KX, int KY, bool MASS>
__device__ __forceinline__ void lens_step_f32(const float* __restrict__ wl, int k,
                                              const float (&ox)[KX], const float (&oy)[KY],
                                              float (&p1)[KX * KY], float (&p2)[KX * KY]) {
    static_assert(KY % 2 == 0, "rays are paired along x2");
    constexpr int R = KX * KY;
    constexpr int G = R > 16 ? 16 : R;
    const LensTerms<KX, KY, MASS> T(wl, k, ox, oy);
#pragma unroll
    for (int g0 = 0; g0 < R; g0 += G) {
        float r2[G], q[G / 2];
#pragma unroll
        for (int t = 0; t < G; ++t) {
            const int r = g0 + t, a = r / KY, b = r % KY;
            r2[t] = __builtin_fmaf(T.dx[a], T.dx[a], T.dy2[b]);
        }
#pragma unroll
        for (int u = 0; u < G / 2; ++u) q[u] = r2[2 * u] * r2[2 * u + 1];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < G / 2; ++u) q[u] = __builtin_amdgcn_rcpf(q[u]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < G / 2; ++u) {
            const int r = g0 + 2 * u, a = r / KY, b = r % KY;
            const float ia = r2[2 * u + 1] * q[u];
            const float ib = r2[2 * u] * q[u];
            p1[r] = __builtin_fmaf(T.dx[a], ia, p1[r]);
            p2[r] = __builtin_fmaf(T.dy[b], ia, p2[r]);
            p1[r + 1] = __builtin_fmaf(T.dx[a], ib, p1[r + 1]);
            p2[r + 1] = __builtin_fmaf(T.dy[b + 1], ib, p2[r + 1]);
        }
    }
}

// One reciprocal per ray, applied only to the pairs flagged in `redo` (bit u
// = rays 2u and 2u + 1).
template <int KX, int KY, bool MASS>
__device__ __forceinline__ void lens_step_f32_single(const float* __restrict__ wl, int k,
                                                     const float (&ox)[KX], const float (&oy)[KY],
                                                     float (&p1)[KX * KY], float (&p2)[KX * KY],
                                                     unsigned redo) {
    constexpr int R = KX * KY;
    const LensTerms<KX, KY, MASS> T(wl, k, ox, oy);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int a = r / KY, b = r % KY;
        const float inv = __builtin_amdgcn_rcpf(__builtin_fmaf(T.dx[a], T.dx[a], T.dy2[b]));
        if ((redo >> (r / 2)) & 1u) {
            p1[r] = __builtin_fmaf(T.dx[a], inv, p1[r]);
            p2[r] = __builtin_fmaf(T.dy[b], inv, p2[r]);
        }
    }
}

// Lens loads each lane keeps in flight while staging a tile (two: deeper
// staging raised the register count of the 16-ray shapes and ran slower).
constexpr int kStageDepth = 2;

// FP32-compensated deflection of the cell's rays; alpha returned in FP64 as
// sum + compensation. With CPW cells per wave, each cell is handled by
// kLanes / CPW lanes (cl = lane within the cell) and has its own rebased copy
// of the lens tile at wl + half * L entries.
template <int KX, int KY, bool MASS, int CPW>
__device__ __forceinline__ void deflect_f32(const MapParams& P, int64_t i0, int64_t j0, int cl,
                                            int half, int L, float* __restrict__ wl,
                                            double (&al1)[KX * KY], double (&al2)[KX * KY]) {
    constexpr int R = KX * KY;
    constexpr int LPC = kLanes / CPW;
    const int lanes_x = P.cx / KX;
    const int lxi = cl % lanes_x, lyi = cl / lanes_x;
    float* __restrict__ wh = wl + (size_t)half * L * (MASS ? 4 : 2);
    // cell centre (a grid line between rays): C = base + (i0 + cx/2) d
    const double C1 = P.base1 + (double)(i0 + P.cx / 2) * P.d1;
    const double C2 = P.base2 + (double)(j0 + P.cy / 2) * P.d2;
    const float C1h = (float)C1, C1l = (float)(C1 - (double)C1h);
    const float C2h = (float)C2, C2l = (float)(C2 - (double)C2h);
    // ray offsets from the cell centre: (half-integer) * d, one FP32 rounding
    float ox[KX], oy[KY];
#pragma unroll
    for (int a = 0; a < KX; ++a) ox[a] = ((float)(lxi * KX + a - P.cx / 2) + 0.5f) * P.d1f;
#pragma unroll
    for (int b = 0; b < KY; ++b) oy[b] = ((float)(lyi * KY + b - P.cy / 2) + 0.5f) * P.d2f;

    float p1[R], p2[R], s1[R], s2[R], c1[R], c2[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { p1[r] = p2[r] = s1[r] = s2[r] = c1[r] = c2[r] = 0.0f; }

    const int64_t n = P.n_lens;
    for (int64_t t0 = 0; t0 < n; t0 += L) {
        const int cnt = (int)((n - t0) < (int64_t)L ? (n - t0) : (int64_t)L);
        // kStageDepth lens loads in flight per lane before the first is
        // used: one load at a time left every wave of the workgroup waiting
        // a full L2 round trip per LPC lenses of the tile
        for (int q0 = cl; q0 < cnt; q0 += LPC * kStageDepth) {
            float4 h[kStageDepth];
            float im[kStageDepth];
#pragma unroll
            for (int u = 0; u < kStageDepth; ++u) {
                const int q = q0 + u * LPC;
                if (q < cnt) {
                    h[u] = P.lens32[t0 + q];
                    if constexpr (MASS) im[u] = P.imass32[t0 + q];
                }
            }
#pragma unroll
            for (int u = 0; u < kStageDepth; ++u) {
                const int q = q0 + u * LPC;
                if (q < cnt) {
                    const float r1 = rebase(h[u].x, h[u].y, C1h, C1l);
                    const float r2 = rebase(h[u].z, h[u].w, C2h, C2l);
                    if constexpr (MASS) {
                        // a massless lens (inverse 0) is staged 2^62 away in
                        // both coordinates: r'^2 products overflow, the shared
                        // reciprocal is 0 and its terms are exactly zero
                        reinterpret_cast<float4*>(wh)[q] =
                            im[u] != 0.0f ? make_float4(r1 * im[u], r2 * im[u], im[u], 0.0f)
                                          : make_float4(-0x1p62f, -0x1p62f, 0.0f, 0.0f);
                    } else {
                        reinterpret_cast<float2*>(wh)[q] = make_float2(r1, r2);
                    }
                }
            }
        }
        __syncthreads();
        for (int b0 = 0; b0 < cnt; b0 += kBlock) {
            const int bn = (cnt - b0) < kBlock ? (cnt - b0) : kBlock;
            if (bn == kBlock) {
                // measured on gfx950: unit masses run fastest with the lens
                // loop unrolled once, mass-weighted lenses with two steps
#pragma unroll(MASS ? 2 : 1)
                for (int k = 0; k < kBlock; ++k) lens_step_f32<KX, KY, MASS>(wh, b0 + k, ox, oy, p1, p2);
            } else {
                for (int k = 0; k < bn; ++k) lens_step_f32<KX, KY, MASS>(wh, b0 + k, ox, oy, p1, p2);
            }
            // Pairs whose block sums are not finite (a ray on a lens, or r^2
            // products beyond the FP32 range) redo the block unpaired.
            unsigned redo = 0;
#pragma unroll
            for (int u = 0; u < R / 2; ++u) {
                const float t = (p1[2 * u] + p2[2 * u]) + (p1[2 * u + 1] + p2[2 * u + 1]);
                if (!__builtin_isfinite(t)) redo |= 1u << u;
            }
            if (__any(redo != 0)) {
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if ((redo >> (r / 2)) & 1u) { p1[r] = 0.0f; p2[r] = 0.0f; }
                for (int k = 0; k < bn; ++k)
                    lens_step_f32_single<KX, KY, MASS>(wh, b0 + k, ox, oy, p1, p2, redo);
            }
            // TwoSum of the running sum and the block sum; the rounding error
            // goes to the compensation term.
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float t = s1[r] + p1[r];
                float bb = t - s1[r];
                c1[r] += (s1[r] - (t - bb)) + (p1[r] - bb);
                s1[r] = t;
                t = s2[r] + p2[r];
                bb = t - s2[r];
                c2[r] += (s2[r] - (t - bb)) + (p2[r] - bb);
                s2[r] = t;
                p1[r] = 0.0f;
                p2[r] = 0.0f;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        al1[r] = (double)s1[r] + (double)c1[r];
        al2[r] = (double)s2[r] + (double)c2[r];
    }
}

// Plain FP64 deflection in the order of a sequential evaluation of eq. 1:
// d = x - x_k; r2 = d1*d1 + d2*d2; q = m / r2; alpha += q * d (no contraction).
template <int KX, int KY, bool MASS>
__device__ __forceinline__ void deflect_f64(const MapParams& P, int64_t i0, int64_t j0, int lane,
                                            int L, double* __restrict__ wl,
                                            double (&al1)[KX * KY], double (&al2)[KX * KY]) {
    constexpr int R = KX * KY;
    const int lanes_x = P.cx / KX;
    const int lxi = lane % lanes_x, lyi = lane / lanes_x;
    double x1[KX], x2[KY];
#pragma unroll
    for (int a = 0; a < KX; ++a) x1[a] = P.base1 + ((double)(i0 + lxi * KX + a) + 0.5) * P.d1;
#pragma unroll
    for (int b = 0; b < KY; ++b) x2[b] = P.base2 + ((double)(j0 + lyi * KY + b) + 0.5) * P.d2;
#pragma unroll
    for (int r = 0; r < R; ++r) { al1[r] = 0.0; al2[r] = 0.0; }

    const int64_t n = P.n_lens;
    for (int64_t t0 = 0; t0 < n; t0 += L) {
        const int cnt = (int)((n - t0) < (int64_t)L ? (n - t0) : (int64_t)L);
        for (int q = lane; q < cnt; q += kLanes) {
            if constexpr (MASS) {
                reinterpret_cast<double4*>(wl)[q] =
                    make_double4(P.lx1[t0 + q], P.lx2[t0 + q], P.lm ? P.lm[t0 + q] : 1.0, 0.0);
            } else {
                reinterpret_cast<double2*>(wl)[q] = make_double2(P.lx1[t0 + q], P.lx2[t0 + q]);
            }
        }
        __syncthreads();
#pragma unroll 2
        for (int k = 0; k < cnt; ++k) {
            double lx, ly, lm = 1.0;
            if constexpr (MASS) {
                const double4 v = reinterpret_cast<const double4*>(wl)[k];
                lx = v.x; ly = v.y; lm = v.z;
            } else {
                const double2 v = reinterpret_cast<const double2*>(wl)[k];
                lx = v.x; ly = v.y;
            }
            double d1[KX], q1[KX], d2[KY], q2[KY];
#pragma unroll
            for (int a = 0; a < KX; ++a) { d1[a] = x1[a] - lx; q1[a] = d1[a] * d1[a]; }
#pragma unroll
            for (int b = 0; b < KY; ++b) { d2[b] = x2[b] - ly; q2[b] = d2[b] * d2[b]; }
#pragma unroll
            for (int a = 0; a < KX; ++a) {
#pragma unroll
                for (int b = 0; b < KY; ++b) {
                    const double r2 = q1[a] + q2[b];
                    const double q = lm / r2;
                    al1[a * KY + b] = al1[a * KY + b] + q * d1[a];
                    al2[a * KY + b] = al2[a * KY + b] + q * d2[b];
                }
            }
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------
// one cell per wave: deflection, lens equation, binning
// ----------------------------------------------------------------------------

// cell and valid are per lane: with CPW cells per wave, lanes
// [h kLanes / CPW, (h + 1) kLanes / CPW) work on cell h of the wave's CPW cells.
template <int KX, int KY, bool MASS, int SUBMAP, bool OUT_Y, int PREC, int CPW>
__device__ __forceinline__ void process_cell(const MapParams& P, int64_t cell, bool valid,
                                             int wave, int lane, int L, char* lens_base,
                                             int* sub, int* hdr) {
    constexpr int R = KX * KY;
    constexpr int LPC = kLanes / CPW;
    const int half = lane / LPC, cl = lane % LPC;
    const int64_t col = cell % P.cells_x;
    const int64_t row = P.cell_row0 + cell / P.cells_x;
    const int64_t i0 = col * P.cx, j0 = row * P.cy;

    double al1[R], al2[R];
    if constexpr (PREC == kFP32Comp) {
        const int stride = MASS ? 16 : 8;
        deflect_f32<KX, KY, MASS, CPW>(P, i0, j0, cl, half, L,
                                       reinterpret_cast<float*>(lens_base + (size_t)wave * CPW * L * stride),
                                       al1, al2);
    } else {
        const int stride = MASS ? 32 : 16;
        deflect_f64<KX, KY, MASS>(P, i0, j0, cl, L,
                                  reinterpret_cast<double*>(lens_base + (size_t)wave * L * stride),
                                  al1, al2);
    }

    const int lanes_x = P.cx / KX;
    const int lxi = cl % lanes_x, lyi = cl / lanes_x;
    int ixs[R], iys[R];
    int esc = 0;
#pragma unroll
    for (int a = 0; a < KX; ++a) {
#pragma unroll
        for (int b = 0; b < KY; ++b) {
            const int r = a * KY + b;
            const int64_t i = i0 + lxi * KX + a;
            const int64_t j = j0 + lyi * KY + b;
            const bool live = valid && i < P.n1 && j >= P.row_begin && j < P.row_end;
            const double x1 = P.base1 + ((double)i + 0.5) * P.d1;
            const double x2 = P.base2 + ((double)j + 0.5) * P.d2;
            const double y1 = P.a1 * x1 - al1[r];
            const double y2 = P.a2 * x2 - al2[r];
            if constexpr (OUT_Y) {
                if (live) {
                    const int64_t o = (j - P.row_begin) * P.n1 + i;
                    P.out_y1[o] = y1;
                    P.out_y2[o] = y2;
                }
                ixs[r] = -1;
                iys[r] = 0;
            } else {
                const double u1 = (y1 - P.lo1) * P.inv1;
                const double u2 = (y2 - P.lo2) * P.inv2;
                const bool in = u1 >= 0.0 && u1 < (double)P.p1 && u2 >= 0.0 && u2 < (double)P.p2;
                // convert only values known to be in range
                const double v1 = in ? u1 : 0.0;
                const double v2 = in ? u2 : 0.0;
                ixs[r] = (live && in) ? (int)v1 : -1;
                iys[r] = (live && in) ? (int)v2 : 0;
                esc += (live && !in) ? 1 : 0;
            }
        }
    }
    if constexpr (OUT_Y) return;

    // Escaped rays: one device atomic per wave on a single address
    // serialised short launches, so the sub-map modes sum them per workgroup
    // in the header first and add them once, after the flush.
    esc = wave_sum(esc);
    if (lane == 0 && esc) {
        if constexpr (SUBMAP) atomicAdd(&hdr[8], esc);
        else atomicAdd(P.escaped, (unsigned long long)esc);
    }

    if constexpr (!SUBMAP) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (ixs[r] >= 0) atomicAdd(P.counts + (int64_t)iys[r] * P.p1 + ixs[r], 1);
    } else {
        // Workgroup-wide sub-map over the bounding box of the binned rays (or,
        // when the box is too large, a kSub x kSub window around their mean
        // pixel, clamped to the box). Rays outside it go straight to global.
        int sx = 0, sy = 0, sc = 0, mnx = INT_MAX, mny = INT_MAX, mxx = -1, mxy = -1;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (ixs[r] >= 0) {
                sx += ixs[r]; sy += iys[r]; sc += 1;
                mnx = min(mnx, ixs[r]); mxx = max(mxx, ixs[r]);
                mny = min(mny, iys[r]); mxy = max(mxy, iys[r]);
            }
        }
        sx = wave_sum(sx);
        sy = wave_sum(sy);
        sc = wave_sum(sc);
        mnx = wave_min(mnx); mny = wave_min(mny);
        mxx = wave_max(mxx); mxy = wave_max(mxy);
        if (lane == 0 && sc) {
            atomicAdd(&hdr[0], sx);
            atomicAdd(&hdr[1], sy);
            atomicAdd(&hdr[2], sc);
            atomicMin(&hdr[4], mnx);
            atomicMin(&hdr[5], mny);
            atomicMax(&hdr[6], mxx);
            atomicMax(&hdr[7], mxy);
        }
        __syncthreads();
        const int cnt = hdr[2];
        if (cnt > 0) {  // uniform across the workgroup
            const int bx0 = hdr[4], by0 = hdr[5];
            const int bw = hdr[6] - bx0 + 1, bh = hdr[7] - by0 + 1;
            int ox = bx0, oy = by0, sw = bw, sh = bh;
            if (SUBMAP == 2 || (int64_t)bw * bh > kSub * kSub) {
                sw = min(bw, kSub);
                sh = min(bh, kSub);
                ox = min(max(hdr[0] / cnt - sw / 2, bx0), bx0 + bw - sw);
                oy = min(max(hdr[1] / cnt - sh / 2, by0), by0 + bh - sh);
            }
            if (SUBMAP == 2) sw = kSub;      // fixed row stride: no division below
            const int area = sw * sh;
            for (int e = threadIdx.x; e < area; e += blockDim.x) sub[e] = 0;
            __syncthreads();
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (ixs[r] >= 0) {
                    const unsigned dx = (unsigned)(ixs[r] - ox), dy = (unsigned)(iys[r] - oy);
                    if (dx < (unsigned)sw && dy < (unsigned)sh)
                        atomicAdd(&sub[dy * sw + dx], 1);
                    else
                        atomicAdd(P.counts + (int64_t)iys[r] * P.p1 + ixs[r], 1);
                }
            }
            __syncthreads();
            for (int e = threadIdx.x; e < area; e += blockDim.x) {
                const int v = sub[e];
                if (v) {
                    const int ey = SUBMAP == 2 ? e / kSub : e / sw;
                    const int ex = SUBMAP == 2 ? e % kSub : e - ey * sw;
                    atomicAdd(P.counts + (int64_t)(oy + ey) * P.p1 + (ox + ex), v);
                }
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const int e = hdr[8];
            if (e) atomicAdd(P.escaped, (unsigned long long)e);
            reset_header(hdr);
        }
        __syncthreads();
    }
}

constexpr int kHdrBytes = 64;

// Occupancy floor in waves per SIMD: 2 holds the 32-ray shapes to 256
// registers; the 16-ray FP32 shapes are held at 3, where they fit without
// spilling (left to itself the compiler gives the unit-mass ones 2 once the
// tile staging keeps two loads in flight; measured on gfx950, 4 with a few
// spilled registers ran ~1 % slower with masses).
template <bool MASS, int CPW, int PREC>
constexpr int min_waves() { return (CPW == 1 && PREC == kFP32Comp) ? 3 : 2; }
template <int KX, int KY, bool MASS, int SUBMAP, bool OUT_Y, int PREC, int CPW>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(min_waves<MASS, CPW, PREC>())))
shoot_kernel(MapParams P, int L) {
    extern __shared__ __align__(16) char smem[];
    int* hdr = reinterpret_cast<int*>(smem);
    char* lens_base = smem + kHdrBytes;
    int* sub = reinterpret_cast<int*>(smem + kHdrBytes);
    if (threadIdx.x == 0) reset_header(hdr);
    __syncthreads();
    const int wave = threadIdx.x / kLanes, lane = threadIdx.x % kLanes;
    const int W = blockDim.x / kLanes;
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t cell = (b * W + wave) * CPW + lane / (kLanes / CPW);
    const bool valid = cell < P.n_cells;
    process_cell<KX, KY, MASS, SUBMAP, OUT_Y, PREC, CPW>(P, valid ? cell : 0, valid, wave, lane, L,
                                                         lens_base, sub, hdr);
}

// Batched launch: the grid is the concatenation of the workgroups of several
// maps (or row segments of maps), segment i owning blocks
// [first[i], first[i] + span_i) with first[i] a multiple of 8, so that block
// b runs on XCD b % 8 exactly as in a single-map launch and the same
// XCD-aware remap applies within the segment. A workgroup finds its segment
// with one wave-wide comparison per 64 segments, then runs the single-map
// body: nothing is carried across cells, so the lens loop compiles as in
// shoot_kernel. Blocks of the padding to the next multiple of 8 exit at once.
template <int KX, int KY, bool MASS, int SUBMAP, int PREC, int CPW>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(min_waves<MASS, CPW, PREC>())))
shoot_batch_kernel(const MapParams* __restrict__ segs, const int64_t* __restrict__ first, int n_segs,
                   int L) {
    extern __shared__ __align__(16) char smem[];
    int* hdr = reinterpret_cast<int*>(smem);
    char* lens_base = smem + kHdrBytes;
    int* sub = reinterpret_cast<int*>(smem + kHdrBytes);
    if (threadIdx.x == 0) reset_header(hdr);
    __syncthreads();
    const int wave = threadIdx.x / kLanes, lane = threadIdx.x % kLanes;
    const int W = blockDim.x / kLanes;
    const int64_t b = blockIdx.x;
    // segment: the number of segments starting at or before b, minus one
    // (first[] ascends and first[0] = 0)
    int m = -1;
    for (int k0 = 0; k0 < n_segs; k0 += kLanes) {
        const int k = k0 + lane;
        const unsigned long long bal = __ballot(k < n_segs && first[k] <= b);
        m += __popcll(bal);
        if (!((bal >> (kLanes - 1)) & 1ull)) break;
    }
    const MapParams& P = segs[m];
    const int64_t per = (int64_t)W * CPW;
    const int64_t nb = (P.n_cells + per - 1) / per;
    const int64_t r = xcd_remap(b - first[m], (nb + 7) / 8 * 8);
    if (r >= nb) return;
    const int64_t cell = (r * W + wave) * CPW + lane / (kLanes / CPW);
    const bool valid = cell < P.n_cells;
    process_cell<KX, KY, MASS, SUBMAP, false, PREC, CPW>(P, valid ? cell : 0, valid, wave, lane, L,
                                                         lens_base, sub, hdr);
}

// ----------------------------------------------------------------------------
// small kernels
// ----------------------------------------------------------------------------

// FP64 lens coordinates -> FP32 hi/lo splits (hi = nearest float, lo = the
// nearest float of the exact remainder) and FP32 inverse masses, 1/m rounded
// once from FP64; a lens with |m| < 2^-40 is massless (inverse 0).
__global__ void prep_lenses_kernel(const double* __restrict__ x1, const double* __restrict__ x2,
                                   const double* __restrict__ m, int64_t n, float4* __restrict__ xy,
                                   float* __restrict__ mo, int write_unit) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const double a = x1[k], b = x2[k];
        const float ah = (float)a, bh = (float)b;
        xy[k] = make_float4(ah, (float)(a - (double)ah), bh, (float)(b - (double)bh));
        if (mo) {
            const double mk = m ? m[k] : (write_unit ? 1.0 : 0.0);
            mo[k] = fabs(mk) >= 0x1p-40 ? (float)(1.0 / mk) : 0.0f;
        }
    }
}

__global__ void bin_positions_kernel(const double* __restrict__ y1, const double* __restrict__ y2,
                                     int64_t n, int32_t p1, int32_t p2, double lo1, double lo2,
                                     double inv1, double inv2, int32_t* __restrict__ counts,
                                     unsigned long long* __restrict__ escaped) {
    int esc = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const double u1 = (y1[k] - lo1) * inv1;
        const double u2 = (y2[k] - lo2) * inv2;
        const bool in = u1 >= 0.0 && u1 < (double)p1 && u2 >= 0.0 && u2 < (double)p2;
        if (in) {
            atomicAdd(counts + (int64_t)(int)u2 * p1 + (int)u1, 1);
        } else {
            esc += 1;
        }
    }
    esc = wave_sum(esc);
    if ((threadIdx.x % kLanes) == 0 && esc) atomicAdd(escaped, (unsigned long long)esc);
}

__global__ void fill_u32_kernel(unsigned int* p, int64_t n, unsigned int v) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
        p[k] = v;
}

int grid_for(int64_t n, int threads, int cap) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// ----------------------------------------------------------------------------
// dispatch
// ----------------------------------------------------------------------------

template <int KX, int KY>
constexpr int cells_per_wave() { return KX * KY / kRaysPerLane; }

// Workgroups per launch: at most kMaxLaunchBlocks. A longer row range goes
// out as several launches over whole cell rows; a cell's rays and lenses do
// not depend on the launch it is in, so no result changes.
constexpr int64_t kMaxBlocks = kMaxLaunchBlocks;

template <int KX, int KY, bool MASS, int SUBMAP, bool OUT_Y, int PREC>
hipError_t launch_one(const MapParams& P, const KernelShape& ks, size_t lds, hipStream_t s) {
    constexpr int CPW = cells_per_wave<KX, KY>();
    const int64_t per_block = (int64_t)ks.waves * CPW;
    if (P.n_cells <= 0) return hipSuccess;
    const int64_t rows = P.n_cells / P.cells_x;   // n_cells covers whole cell rows
    const int64_t rows_per_launch = kMaxBlocks * per_block / P.cells_x;
    if (rows_per_launch < 1 || rows * P.cells_x != P.n_cells) return hipErrorInvalidValue;
    for (int64_t r0 = 0; r0 < rows; r0 += rows_per_launch) {
        MapParams Q = P;
        Q.cell_row0 = P.cell_row0 + r0;
        Q.n_cells = (rows - r0 < rows_per_launch ? rows - r0 : rows_per_launch) * P.cells_x;
        const int64_t blocks = (Q.n_cells + per_block - 1) / per_block;
        hipLaunchKernelGGL((shoot_kernel<KX, KY, MASS, SUBMAP, OUT_Y, PREC, CPW>), dim3((unsigned)blocks),
                           dim3(ks.waves * kLanes), lds, s, Q, ks.lens_tile);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int KX, int KY, bool MASS, int SUBMAP, int PREC>
hipError_t launch_batch_one(const MapParams* segs, const int64_t* first, int n_segs, int64_t blocks,
                            const KernelShape& ks, size_t lds, hipStream_t s) {
    if (blocks <= 0 || n_segs <= 0) return hipSuccess;
    if (blocks > kMaxBlocks) return hipErrorInvalidValue;
    hipLaunchKernelGGL((shoot_batch_kernel<KX, KY, MASS, SUBMAP, PREC, cells_per_wave<KX, KY>()>),
                       dim3((unsigned)blocks), dim3(ks.waves * kLanes), lds, s, segs, first, n_segs,
                       ks.lens_tile);
    return hipGetLastError();
}

template <int KX, int KY, bool MASS, int PREC>
hipError_t dispatch_submap(const MapParams& P, const KernelShape& ks, size_t lds, hipStream_t s) {
    switch (ks.submap) {
        case 1: return launch_one<KX, KY, MASS, 1, false, PREC>(P, ks, lds, s);
        case 2: return launch_one<KX, KY, MASS, 2, false, PREC>(P, ks, lds, s);
        default: return launch_one<KX, KY, MASS, 0, false, PREC>(P, ks, lds, s);
    }
}

template <int KX, int KY, int PREC>
hipError_t dispatch_shape(const MapParams& P, const KernelShape& ks, bool masses, bool out_y,
                          size_t lds, hipStream_t s) {
    if (out_y) {
        return masses ? launch_one<KX, KY, true, 0, true, PREC>(P, ks, lds, s)
                      : launch_one<KX, KY, false, 0, true, PREC>(P, ks, lds, s);
    }
    return masses ? dispatch_submap<KX, KY, true, PREC>(P, ks, lds, s)
                  : dispatch_submap<KX, KY, false, PREC>(P, ks, lds, s);
}

template <int KX, int KY, bool MASS, int PREC>
hipError_t dispatch_batch_submap(const MapParams* segs, const int64_t* first, int n_segs, int64_t blocks,
                                 const KernelShape& ks, size_t lds, hipStream_t s) {
    switch (ks.submap) {
        case 1: return launch_batch_one<KX, KY, MASS, 1, PREC>(segs, first, n_segs, blocks, ks, lds, s);
        case 2: return launch_batch_one<KX, KY, MASS, 2, PREC>(segs, first, n_segs, blocks, ks, lds, s);
        default: return launch_batch_one<KX, KY, MASS, 0, PREC>(segs, first, n_segs, blocks, ks, lds, s);
    }
}

template <int KX, int KY, int PREC>
hipError_t dispatch_batch_shape(const MapParams* segs, const int64_t* first, int n_segs, int64_t blocks,
                                bool masses, const KernelShape& ks, size_t lds, hipStream_t s) {
    return masses ? dispatch_batch_submap<KX, KY, true, PREC>(segs, first, n_segs, blocks, ks, lds, s)
                  : dispatch_batch_submap<KX, KY, false, PREC>(segs, first, n_segs, blocks, ks, lds, s);
}

}  // namespace

bool shape_supported(Precision prec, const KernelShape& ks) {
    const bool k44 = ks.rays_x == 4 && ks.rays_y == 4;
    const bool k28 = ks.rays_x == 2 && ks.rays_y == 8;
    const bool k82 = ks.rays_x == 8 && ks.rays_y == 2;
    const bool k48 = ks.rays_x == 4 && ks.rays_y == 8;   // 32 rays per lane, two cells per wave
    const bool k84 = ks.rays_x == 8 && ks.rays_y == 4;
    if (prec == kFP64Plain && !k44) return false;
    if (!(k44 || k28 || k82 || k48 || k84)) return false;
    if (ks.lens_tile < kBlock || ks.lens_tile > 2048 || ks.lens_tile % kBlock) return false;
    if (!(ks.waves == 1 || ks.waves == 2 || ks.waves == 4)) return false;
    if (ks.submap < 0 || ks.submap > 2) return false;
    return true;
}

// Dynamic LDS per workgroup is kept within 64 KiB: a lens tile that would not
// fit is shrunk (in whole compensation blocks), which changes no result.
constexpr size_t kMaxLds = 65536;

// LDS bytes of one lens entry times the cells per wave (each cell stages its
// own rebased copy).
size_t lens_entry_bytes(Precision prec, bool masses, const KernelShape& ks) {
    const size_t stride = prec == kFP32Comp ? (masses ? 16 : 8) : (masses ? 32 : 16);
    return stride * (size_t)(ks.rays_x * ks.rays_y / kRaysPerLane);
}

KernelShape fit_lds(Precision prec, bool masses, const KernelShape& ks) {
    const size_t stride = lens_entry_bytes(prec, masses, ks);
    KernelShape k = ks;
    const size_t room = kMaxLds - kHdrBytes;
    while (k.lens_tile > kBlock && (size_t)k.waves * k.lens_tile * stride > room) k.lens_tile -= kBlock;
    return k;
}

size_t shoot_lds_bytes(Precision prec, bool masses, const KernelShape& ks) {
    const size_t stride = lens_entry_bytes(prec, masses, ks);
    size_t lens = (size_t)ks.waves * ks.lens_tile * stride;
    const size_t sub = ks.submap ? (size_t)kSub * kSub * sizeof(int) : 0;
    return kHdrBytes + (lens > sub ? lens : sub);
}

hipError_t launch_shoot(const MapParams& P, Precision prec, const KernelShape& ks, bool out_y,
                        int num_cus, hipStream_t s) {
    (void)num_cus;
    const bool masses = prec == kFP32Comp ? (P.imass32 != nullptr) : (P.lm != nullptr);
    KernelShape k = fit_lds(prec, masses, ks);
    if (out_y) k.submap = 0;
    const size_t lds = shoot_lds_bytes(prec, masses, k);
    if (prec == kFP64Plain) return dispatch_shape<4, 4, kFP64Plain>(P, k, masses, out_y, lds, s);
    if (k.rays_x == 4 && k.rays_y == 4) return dispatch_shape<4, 4, kFP32Comp>(P, k, masses, out_y, lds, s);
    if (k.rays_x == 2) return dispatch_shape<2, 8, kFP32Comp>(P, k, masses, out_y, lds, s);
    if (k.rays_x == 4) return dispatch_shape<4, 8, kFP32Comp>(P, k, masses, out_y, lds, s);
    if (k.rays_y == 4) return dispatch_shape<8, 4, kFP32Comp>(P, k, masses, out_y, lds, s);
    return dispatch_shape<8, 2, kFP32Comp>(P, k, masses, out_y, lds, s);
}

int64_t batch_cells_per_block(const KernelShape& ks) {
    return (int64_t)ks.waves * (ks.rays_x * ks.rays_y / kRaysPerLane);
}

hipError_t launch_shoot_batch(const MapParams* d_segs, const int64_t* d_first, int n_segs, int64_t blocks,
                              Precision prec, bool masses, const KernelShape& ks_in, hipStream_t s) {
    const KernelShape ks = fit_lds(prec, masses, ks_in);
    const size_t lds = shoot_lds_bytes(prec, masses, ks);
    if (prec == kFP64Plain)
        return dispatch_batch_shape<4, 4, kFP64Plain>(d_segs, d_first, n_segs, blocks, masses, ks, lds, s);
    if (ks.rays_x == 4 && ks.rays_y == 4)
        return dispatch_batch_shape<4, 4, kFP32Comp>(d_segs, d_first, n_segs, blocks, masses, ks, lds, s);
    if (ks.rays_x == 2)
        return dispatch_batch_shape<2, 8, kFP32Comp>(d_segs, d_first, n_segs, blocks, masses, ks, lds, s);
    if (ks.rays_x == 4)
        return dispatch_batch_shape<4, 8, kFP32Comp>(d_segs, d_first, n_segs, blocks, masses, ks, lds, s);
    if (ks.rays_y == 4)
        return dispatch_batch_shape<8, 4, kFP32Comp>(d_segs, d_first, n_segs, blocks, masses, ks, lds, s);
    return dispatch_batch_shape<8, 2, kFP32Comp>(d_segs, d_first, n_segs, blocks, masses, ks, lds, s);
}

hipError_t launch_prep_lenses(const double* x1, const double* x2, const double* m, int64_t n,
                              float4* out_xy, float* out_m, bool write_unit_mass, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(prep_lenses_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, x1, x2, m,
                       n, out_xy, out_m, write_unit_mass ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_bin_positions(const double* y1, const double* y2, int64_t n, int32_t p1,
                                int32_t p2, double lo1, double lo2, double inv1, double inv2,
                                int32_t* counts, unsigned long long* escaped, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(bin_positions_kernel, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, y1, y2, n,
                       p1, p2, lo1, lo2, inv1, inv2, counts, escaped);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned int* p, int64_t n, unsigned int v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// staging that allocates nothing (rl_shoot_noalloc)
// ----------------------------------------------------------------------------

namespace {

// FP32 lens copies of rl_shoot_noalloc: RL_NOALLOC_MAX_LENSES float4 entries
// {x1 hi, x1 lo, x2 hi, x2 lo}, then as many FP32 inverse masses. Each GPU
// holds its own copy from the library's load until the process ends. Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
constexpr size_t kNoAllocXyBytes = (size_t)RL_NOALLOC_MAX_LENSES * sizeof(float4);
constexpr size_t kNoAllocBytes = kNoAllocXyBytes + (size_t)RL_NOALLOC_MAX_LENSES * sizeof(float);
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_address(int device, unsigned char** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[device]);
    return hipSuccess;
}

}  // namespace

hipError_t launch_shoot_noalloc(MapParams P, const double* x1, const double* x2, const double* m,
                                int64_t n, Precision prec, const KernelShape& ks, int device,
                                hipStream_t s) {
    if (n < 0 || n > RL_NOALLOC_MAX_LENSES) return hipErrorInvalidValue;
    if (prec == kFP32Comp) {
        unsigned char* base = nullptr;
        const hipError_t e = scratch_address(device, &base);
        if (e != hipSuccess) return e;
        float4* xy = reinterpret_cast<float4*>(base);
        float* mf = reinterpret_cast<float*>(base + kNoAllocXyBytes);
        // every entry the shoot kernel reads ([0, n)) is written here first
        const hipError_t e2 = launch_prep_lenses(x1, x2, m, n, xy, m ? mf : nullptr, true, s);
        if (e2 != hipSuccess) return e2;
        P.lens32 = xy;
        P.imass32 = m ? mf : nullptr;
    } else {
        P.lx1 = x1;
        P.lx2 = x2;
        P.lm = m;
    }
    P.n_lens = n;
    return launch_shoot(P, prec, ks, false, 0, s);
}

}  // namespace rl
