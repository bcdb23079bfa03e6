// Internal declarations shared by the ray-shooting kernels (shoot.hip), the
// other kernels and the C-ABI layer (api.cpp) of the raylens library. Not
// part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "raylens.h"

#define RL_TRY(expr)                      \
    do {                                  \
        rl_status st_ = (expr);           \
        if (st_ != RL_OK) return st_;     \
    } while (0)

namespace rl {

// Error reporting shared by the C-ABI sources: sets the calling thread's
// rl_last_error() text (printf-style) and returns st.
rl_status set_error(rl_status st, const char* fmt, ...);
void clear_error();
// HIP device ordinal of a context.
int context_device(const rl_context* ctx);
// Tuning classes: lens-count class 0 (N < 1000), 1 (N < 10000), 2; plus 3
// for lens fields with masses.
constexpr int kTuningClasses = 6;
inline int tuning_class(int64_t n, bool masses) {
    return (n < 1000 ? 0 : (n < 10000 ? 1 : 2)) + (masses ? 3 : 0);
}

// Rays per origin cell and per wave: one wave of 64 lanes holds 16 rays per
// lane. A cell is the unit whose centre the FP32 lens coordinates are
// rebased to; its shape depends only on the ray grid, so no kernel-shape
// knob changes a result bit.
constexpr int kLanes = 64;
constexpr int kRaysPerLane = 16;
constexpr int kCellRays = kLanes * kRaysPerLane;
// Lenses per compensation block: each block is summed in plain FP32 and the
// block sums are added with TwoSum. Fixed, so results do not depend on the
// LDS lens tile.
constexpr int kBlock = 256;
// LDS-privatised sub-map edge (pixels).
constexpr int kSub = 64;

enum Precision : int32_t { kFP32Comp = 0, kFP64Plain = 1 };

// Everything a kernel needs about one map. Built on the host in FP64 with the
// same IEEE operations the method states, passed by value (single map) or
// from device memory (batch).
struct MapParams {
    // ray grid: x = base + (i + 1/2) * d
    int64_t n1, n2;
    double base1, base2, d1, d2;
    float d1f, d2f;
    int32_t cx, cy;            // cell shape in rays, cx * cy = kCellRays
    int64_t cells_x;           // cells along x1 (last one may be partial)
    int64_t row_begin, row_end;
    int64_t cell_row0;         // first cell row touching row_begin
    int64_t n_cells;           // cells covering [row_begin, row_end)
    // macro model: y1 = a1 x1 - alpha1, y2 = a2 x2 - alpha2
    double a1, a2;
    // window: u = (y - lo) * inv; binned iff 0 <= u < p
    int32_t p1, p2;
    double lo1, lo2, inv1, inv2;
    // lenses
    int64_t n_lens;
    const float4* lens32;      // FP32 path: {x1 hi, x1 lo, x2 hi, x2 lo}
    const float* imass32;      // FP32 path inverse masses 1/m (0: massless; nullptr = unit)
    const double* lx1;         // FP64 path
    const double* lx2;
    const double* lm;          // FP64 path masses (nullptr = unit)
    // outputs
    int32_t* counts;
    unsigned long long* escaped;
    double* out_y1;            // per-ray output mode only
    double* out_y2;
};

// Workgroups per launch of the shoot kernels: at most 2^23 (2^31 work-items
// with 4 waves, inside the 32-bit size of one dispatch). The host refuses
// grids wider than 2^26 rays, so one cell row (at most 2^23 cells of >= 8
// rays across) always fits one launch.
constexpr int64_t kMaxLaunchBlocks = (int64_t)1 << 23;

struct KernelShape {
    int32_t rays_x, rays_y;    // rays per lane along x1 / x2 (product 16; 32 = two cells per wave)
    int32_t lens_tile;         // lenses per LDS pass (multiple of kBlock)
    int32_t waves;             // waves per workgroup
    int32_t submap;            // 0 global atomics, 1 bounding-box LDS sub-map, 2 64x64 LDS window
};

// Launchers of shoot.hip. Each returns the hipError_t of the launch. The
// kernels of finished maps and of the convolution are declared in maps.h.
hipError_t launch_prep_lenses(const double* x1, const double* x2, const double* m, int64_t n,
                              float4* out_xy, float* out_m, bool write_unit_mass,
                              hipStream_t stream);
hipError_t launch_shoot(const MapParams& P, Precision prec, const KernelShape& ks, bool out_y,
                        int num_cus, hipStream_t stream);
// Batched launch over n_segs segments (device arrays): segment i is a map, or
// a range of whole cell rows of one, with its workgroups at blocks
// [first[i], first[i] + span_i) of the grid, span_i = the segment's blocks
// (batch_cells_per_block cells each) rounded up to a multiple of 8, first[0]
// = 0, and `blocks` = the sum of the spans, at most kMaxLaunchBlocks.
int64_t batch_cells_per_block(const KernelShape& ks);
hipError_t launch_shoot_batch(const MapParams* d_segs, const int64_t* d_first, int n_segs, int64_t blocks,
                              Precision prec, bool masses, const KernelShape& ks, hipStream_t stream);
hipError_t launch_bin_positions(const double* y1, const double* y2, int64_t n, int32_t p1,
                                int32_t p2, double lo1, double lo2, double inv1, double inv2,
                                int32_t* counts, unsigned long long* escaped, hipStream_t stream);
hipError_t launch_fill_u32(unsigned int* p, int64_t n, unsigned int v, hipStream_t stream);
// rl_shoot_noalloc's staging: the FP32 lens copies of P's lenses (FP64 x1,
// x2, m; n <= RL_NOALLOC_MAX_LENSES, checked by the caller) go to the
// library's fixed per-device array instead of context memory, then P is shot.
// The device must be current.
hipError_t launch_shoot_noalloc(MapParams P, const double* x1, const double* x2, const double* m,
                                int64_t n, Precision prec, const KernelShape& ks, int device,
                                hipStream_t stream);

bool shape_supported(Precision prec, const KernelShape& ks);
size_t shoot_lds_bytes(Precision prec, bool masses, const KernelShape& ks);

}  // namespace rl
