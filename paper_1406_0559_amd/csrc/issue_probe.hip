// FP32 VALU issue rates on gfx950: the ceiling against which the shoot
// kernel's instruction rate is compared (a standalone program, not part of the
// library).
//
// Each lane runs CH independent dependency chains of one instruction kind for
// `iters` iterations; every operand of the plain streams lives in a VGPR
// (an operand from an SGPR or a literal lowers the rate, see the "sgpr" row).
// Workgroups of 256 threads (4 waves), `per` workgroups per CU: `per` waves
// per SIMD when all are resident. The shader clock is read in the kernel (s_memtime) against
// the 100 MHz real-time counter (s_memrealtime), so the rate is per clock at
// the clock the kernel actually ran at. Rates are lane-instructions per CU per
// clock (a wave instruction counts 64).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(x)                                                                     \
    do {                                                                             \
        hipError_t e_ = (x);                                                         \
        if (e_ != hipSuccess) {                                                      \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));             \
            std::exit(1);                                                            \
        }                                                                            \
    } while (0)

enum Mode { kFma = 0, kMul = 1, kAdd = 2, kRcp = 3, kFmaRcp = 4, kFmaSgpr = 5 };

template <int MODE, int CH>
__global__ void __launch_bounds__(256) probe(float* out, int iters, float sa, long long* clk) {
    float x[CH], y[CH], z[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        x[c] = threadIdx.x * 1e-3f + c;
        y[c] = 1.0f + c * 1e-4f + threadIdx.x * 1e-9f;
        z[c] = 0.999f - c * 1e-5f + threadIdx.x * 1e-9f;
    }
    const long long t0 = clock64();
    const long long r0 = __builtin_amdgcn_s_memrealtime();
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            if constexpr (MODE == kFma) x[c] = __builtin_fmaf(x[c], z[c], y[c]);
            else if constexpr (MODE == kMul) x[c] = x[c] * z[c];
            else if constexpr (MODE == kAdd) x[c] = x[c] + z[c];
            else if constexpr (MODE == kRcp) x[c] = __builtin_amdgcn_rcpf(x[c]);
            else if constexpr (MODE == kFmaRcp) {
                if (c % 2 == 0) x[c] = __builtin_fmaf(x[c], z[c], y[c]);
                else x[c] = __builtin_amdgcn_rcpf(x[c]);
            } else {
                x[c] = __builtin_fmaf(x[c], sa, y[c]);
            }
        }
    }
    const long long t1 = clock64();
    const long long r1 = __builtin_amdgcn_s_memrealtime();
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < CH; ++c) s += x[c] + y[c] + z[c];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
    if (threadIdx.x == 0) {
        clk[2 * blockIdx.x] = t1 - t0;
        clk[2 * blockIdx.x + 1] = r1 - r0;
    }
}

template <int MODE, int CH>
void run(const char* name, int cus, int per, int iters, float* d_out, long long* d_clk) {
    const int blocks = cus * per;
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    for (int w = 0; w < 3; ++w)
        hipLaunchKernelGGL((probe<MODE, CH>), dim3(blocks), dim3(256), 0, 0, d_out, iters, 0.999f, d_clk);
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    CHECK(hipEventRecord(e0));
    hipLaunchKernelGGL((probe<MODE, CH>), dim3(blocks), dim3(256), 0, 0, d_out, iters, 0.999f, d_clk);
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    float ms = 0.0f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    std::vector<long long> clk(2 * (size_t)blocks);
    CHECK(hipMemcpy(clk.data(), d_clk, clk.size() * sizeof(long long), hipMemcpyDeviceToHost));
    double cyc = 0.0, real = 0.0;
    for (int b = 0; b < blocks; ++b) {
        cyc += (double)clk[2 * b];
        real += (double)clk[2 * b + 1];
    }
    const double ghz = cyc / (real / 100e6) / 1e9;
    const double lanes = (double)blocks * 4 * iters * CH * 64;
    std::printf("%-8s %2d waves/SIMD  %8.3f ms  %.3f GHz  %6.1f lane-instr/CU/clk\n", name, per, ms, ghz,
                lanes / (ms * 1e-3) / cus / (ghz * 1e9));
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
}

int main() {
    int cus = 0;
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
    const int max_per = 8;
    float* d_out = nullptr;
    long long* d_clk = nullptr;
    CHECK(hipMalloc(&d_out, (size_t)cus * max_per * 256 * sizeof(float)));
    CHECK(hipMalloc(&d_clk, (size_t)2 * cus * max_per * sizeof(long long)));
    std::printf("%d CUs; 16 independent chains per lane\n", cus);
    for (int per : {1, 2, 3, 4, 8}) run<kFma, 16>("fma", cus, per, 100000, d_out, d_clk);
    run<kMul, 16>("mul", cus, 3, 100000, d_out, d_clk);
    run<kAdd, 16>("add", cus, 3, 100000, d_out, d_clk);
    run<kRcp, 16>("rcp", cus, 3, 25000, d_out, d_clk);
    run<kFmaRcp, 16>("fma:rcp", cus, 3, 50000, d_out, d_clk);
    run<kFmaSgpr, 16>("sgpr", cus, 3, 100000, d_out, d_clk);
    CHECK(hipFree(d_out));
    CHECK(hipFree(d_clk));
    return 0;
}
