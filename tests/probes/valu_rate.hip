// Issue rate of wave64 VALU instructions on one GPU: cycles per instruction
// per SIMD, at the 2.4 GHz peak engine clock, for FP32 FMA, FP32 ADD, a
// 32-bit integer XOR and FP64 FMA, with 1, 2, 4 and 8 waves per SIMD.
//
// Each lane runs 8 independent register chains of one instruction kind (the
// instructions are written in inline assembly so that the loop holds exactly
// 8 of them per iteration), so a SIMD's rate is limited by issue, not by the
// latency of one chain.  Every kernel runs for milliseconds, after 300 ms of
// the same work untimed: the clock settles under sustained load.  Grid: 256
// workgroups of 256 threads (one wave per SIMD of every CU) per wave per SIMD.
#include <hip/hip_runtime.h>
#include <chrono>
#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                                          \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess) {                                                           \
            fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));                \
            exit(1);                                                                      \
        }                                                                                 \
    } while (0)

enum Kind { FMA_F32, ADD_F32, XOR_B32, FMA_F64, N_KINDS };
static const char* kKindName[N_KINDS] = {"v_fmac_f32", "v_add_f32", "v_xor_b32", "v_fma_f64"};

template <int KIND>
__global__ void __launch_bounds__(256) issue(float* out, int n_it, float b, float c, int k) {
    float a[8];
    double d[8];
    int x[8];
    for (int j = 0; j < 8; ++j) {
        a[j] = threadIdx.x * 1e-3f + j;
        d[j] = a[j];
        x[j] = threadIdx.x + j;
    }
    const double bd = b, cd = c;
    for (int it = 0; it < n_it; ++it) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (KIND == FMA_F32) asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(a[j]) : "v"(b), "v"(c));
            if (KIND == ADD_F32) asm volatile("v_add_f32 %0, %0, %1" : "+v"(a[j]) : "v"(b));
            if (KIND == XOR_B32) asm volatile("v_xor_b32 %0, %0, %1" : "+v"(x[j]) : "v"(k));
            if (KIND == FMA_F64) asm volatile("v_fma_f64 %0, %0, %1, %2" : "+v"(d[j]) : "v"(bd), "v"(cd));
        }
    }
    float s = 0.0f;
    for (int j = 0; j < 8; ++j) s += a[j] + (float)d[j] + (float)x[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

static int g_cus = 0;

// cycles per wave-instruction per SIMD at 2.4 GHz for one launch
static double run(int kind, int waves, int n_it, float* out) {
    const dim3 grid(g_cus * waves), block(256);
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    CHECK(hipEventRecord(e0));
    switch (kind) {
        case FMA_F32: hipLaunchKernelGGL(issue<FMA_F32>, grid, block, 0, 0, out, n_it, 1.0000001f, 1e-7f, 3); break;
        case ADD_F32: hipLaunchKernelGGL(issue<ADD_F32>, grid, block, 0, 0, out, n_it, 1.0000001f, 1e-7f, 3); break;
        case XOR_B32: hipLaunchKernelGGL(issue<XOR_B32>, grid, block, 0, 0, out, n_it, 1.0000001f, 1e-7f, 3); break;
        default: hipLaunchKernelGGL(issue<FMA_F64>, grid, block, 0, 0, out, n_it, 1.0000001f, 1e-7f, 3); break;
    }
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    float ms = 0.0f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    const double per_simd = (double)n_it * 8 * waves;   // wave-instructions per SIMD
    return ms * 1e-3 * 2.4e9 / per_simd;
}

int main() {
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0));
    g_cus = prop.multiProcessorCount;
    const int max_waves = 8;
    float* out = nullptr;
    CHECK(hipMalloc(&out, sizeof(float) * (size_t)g_cus * max_waves * 256));
    const auto t0 = std::chrono::steady_clock::now();
    while (std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() < 0.3)
        run(FMA_F32, max_waves, 20000, out);
    printf("device %s, %d compute units; cycles per wave64 instruction per SIMD at 2.4 GHz\n", prop.name, g_cus);
    printf("%-12s %8s %8s %8s %8s\n", "instruction", "1 wave", "2 waves", "4 waves", "8 waves");
    for (int kind = 0; kind < N_KINDS; ++kind) {
        printf("%-12s", kKindName[kind]);
        for (int w : {1, 2, 4, 8}) {
            double best = 1e30;
            for (int rep = 0; rep < 2; ++rep) {
                const double c = run(kind, w, 40000, out);
                best = c < best ? c : best;
            }
            printf(" %8.2f", best);
        }
        printf("\n");
        fflush(stdout);
    }
    CHECK(hipFree(out));
    return 0;
}
