// valu_rates -- issue rates of single VALU instruction forms on gfx950, the
// measurements behind the force kernels' FP32 ceiling.
//
// Each kernel runs a stream of one instruction form on 8 independent
// accumulators per thread (or a fixed mix), blocks of 256 threads, 1, 2, 4
// or 8 blocks per compute unit (that many waves per SIMD).  Reported per
// form and occupancy: lane operations per clock per CU, at the shader clock
// the waves measured themselves (s_memtime against the 100 MHz constant
// counter s_memrealtime), and lane operations per second.  A CU has four
// SIMDs of 16 lanes; 64 lane-operations per clock is one instruction per
// SIMD per cycle, 128 is two (instructions of different waves issued
// together).
//
//   valu_rates            (prints one line per form and occupancy)
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(x)                                                                   \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));           \
            std::exit(1);                                                          \
        }                                                                          \
    } while (0)

#define R8(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7)

template <int K>
__device__ __forceinline__ void body(float (&a)[8], float b, float c)
{
#define FMAC(i) asm volatile("v_fmac_f32_e32 %0, %1, %2" : "+v"(a[i]) : "v"(b), "v"(c));
#define FMA3(i) asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(a[i]) : "v"(b), "v"(c));
#define MUL2(i) asm volatile("v_mul_f32_e32 %0, %1, %0" : "+v"(a[i]) : "v"(b));
#define ADD2(i) asm volatile("v_add_f32_e32 %0, %1, %0" : "+v"(a[i]) : "v"(b));
#define RSQ(i) asm volatile("v_rsq_f32_e32 %0, %0" : "+v"(a[i]));
    if constexpr (K == 0) { R8(FMAC) }
    if constexpr (K == 1) { R8(FMA3) }
    if constexpr (K == 2) { R8(MUL2) }
    if constexpr (K == 3) { R8(ADD2) }
    if constexpr (K == 4) { R8(RSQ) }
    if constexpr (K == 5) { R8(FMAC) RSQ(0) }
    if constexpr (K == 6) { FMAC(0) FMA3(1) FMAC(2) MUL2(3) FMAC(4) FMA3(5) FMAC(6) MUL2(7) }
#undef FMAC
#undef FMA3
#undef MUL2
#undef ADD2
#undef RSQ
}
constexpr int kInstr[] = {8, 8, 8, 8, 8, 9, 8};
const char *kName[] = {"v_fmac_f32 (VOP2)", "v_fma_f32 (VOP3)", "v_mul_f32", "v_add_f32",
                       "v_rsq_f32", "8 fmac + 1 rsq", "fmac/fma/mul mix"};

template <int K>
__global__ __launch_bounds__(256) void probe(float *out, unsigned long long *cyc, int iters)
{
    float a[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = 1.0f + 1e-3f * (threadIdx.x + i);
    const float b = 0.99999f + 1e-9f * threadIdx.x, c = 1e-7f;
    const unsigned long long t0 = __builtin_amdgcn_s_memtime();
    const unsigned long long r0 = __builtin_amdgcn_s_memrealtime();
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 8; ++u) body<K>(a, b, c);
    }
    const unsigned long long t1 = __builtin_amdgcn_s_memtime();
    const unsigned long long r1 = __builtin_amdgcn_s_memrealtime();
    float s = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) s += a[i];
    out[blockIdx.x * 256 + threadIdx.x] = s;
    if ((threadIdx.x & 63) == 0) {
        const int w = blockIdx.x * 4 + threadIdx.x / 64;
        cyc[2 * w] = t1 - t0;
        cyc[2 * w + 1] = r1 - r0;
    }
}

template <int K>
void run(int blocks_per_cu, int ncu, float *out, unsigned long long *cyc, int iters)
{
    const int grid = blocks_per_cu * ncu;
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    hipLaunchKernelGGL(probe<K>, dim3(grid), dim3(256), 0, 0, out, cyc, iters);  // warm-up
    CHECK(hipEventRecord(e0, 0));
    hipLaunchKernelGGL(probe<K>, dim3(grid), dim3(256), 0, 0, out, cyc, iters);
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipEventSynchronize(e1));
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    std::vector<unsigned long long> h(2 * (size_t)grid * 4);
    CHECK(hipMemcpy(h.data(), cyc, h.size() * 8, hipMemcpyDeviceToHost));
    double cs = 0, rs = 0;
    for (int w = 0; w < grid * 4; ++w) {
        cs += (double)h[2 * w];
        rs += (double)h[2 * w + 1];
    }
    const double clk_ghz = cs / (rs * 10.0);  // s_memrealtime counts at 100 MHz
    const double lane_ops = (double)iters * 8 * kInstr[K] * 64.0 * grid * 4;
    std::printf("%-20s waves/SIMD %d: clock %.3f GHz, kernel %.3f ms, %.1f lane-ops/clk/CU, "
                "%.0f Glane-ops/s\n",
                kName[K], blocks_per_cu, clk_ghz, ms,
                lane_ops / (ms * 1e-3 * clk_ghz * 1e9) / ncu, lane_ops / (ms * 1e-3) / 1e9);
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
}

template <int K>
void sweep(int ncu, float *out, unsigned long long *cyc)
{
    for (int w : {1, 2, 4, 8}) run<K>(w, ncu, out, cyc, 4096);
}

int main()
{
    hipDeviceProp_t p;
    CHECK(hipGetDeviceProperties(&p, 0));
    const int ncu = p.multiProcessorCount;
    std::printf("device %s, %d CUs\n", p.gcnArchName, ncu);
    float *out;
    unsigned long long *cyc;
    CHECK(hipMalloc(&out, (size_t)8 * ncu * 256 * sizeof(float)));
    CHECK(hipMalloc(&cyc, (size_t)8 * ncu * 4 * 2 * sizeof(unsigned long long)));
    sweep<0>(ncu, out, cyc);
    sweep<1>(ncu, out, cyc);
    sweep<2>(ncu, out, cyc);
    sweep<3>(ncu, out, cyc);
    sweep<4>(ncu, out, cyc);
    sweep<5>(ncu, out, cyc);
    sweep<6>(ncu, out, cyc);
    CHECK(hipFree(out));
    CHECK(hipFree(cyc));
    return 0;
}
