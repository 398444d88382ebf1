// interaction_rates -- throughput of the force kernels' interaction terms
// (bhq_terms.h: the particle term and the quadrupole cell term, FP32) with
// nothing else around them: the arithmetic ceiling of the force kernels on
// gfx950.  Each thread owns IB i-particles and goes over 64 list entries,
// read from registers or as LDS broadcasts (as the kernels read them),
// 200 times; blocks of 256 threads, 2, 4, 6 or 8 blocks per compute unit
// (waves per SIMD).  Reported: interactions per second and hardware-counted
// FP32 TFLOP/s (20 flops per particle term, 53 per cell term; FMA = 2,
// rsqrt = 1) and their fraction of the 157.3 TFLOP/s FP32 vector peak; the
// shader clock the waves measured (s_memtime against the 100 MHz
// s_memrealtime); and the terms' VALU instructions (14 per particle term,
// 34 per cell term, rsqrt counted once) issued per SIMD per quad-cycle
// (4 clocks: at most 2, two waves' instructions together), the rate to
// compare with a force kernel's counters.
//
//   interaction_rates
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../csrc/bhq_terms.h"

#define CHECK(x)                                                                   \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));           \
            std::exit(1);                                                          \
        }                                                                          \
    } while (0)

using bhq::V4;

// MODE 0: cell term, entries in registers; 1: cell term from LDS;
// 2: particle term in registers; 3: particle term from LDS
template <int MODE, int IB>
__global__ __launch_bounds__(256) void body(float *out, unsigned long long *cyc, int iters,
                                            const V4<float> *src)
{
    __shared__ V4<float> sa[64], sb[64], sc[64];
    const int t = threadIdx.x;
    if (t < 64) {
        sa[t] = src[t];
        sb[t] = src[64 + t];
        sc[t] = src[128 + t];
    }
    __syncthreads();
    float xi[IB], yi[IB], zi[IB], ax[IB], ay[IB], az[IB], pt[IB];
    for (int u = 0; u < IB; ++u) {
        xi[u] = 0.01f * (t + u);
        yi[u] = 0.02f * u;
        zi[u] = -0.01f * t;
        ax[u] = ay[u] = az[u] = pt[u] = 0.0f;
    }
    const float e2 = 1e-4f;
    const V4<float> ra = src[t & 63], rb = src[64 + (t & 63)], rc = src[128 + (t & 63)];
    const unsigned long long c0 = __builtin_amdgcn_s_memtime();
    const unsigned long long r0 = __builtin_amdgcn_s_memrealtime();
    for (int it = 0; it < iters; ++it) {
#pragma unroll 2
        for (int k = 0; k < 64; ++k) {
            V4<float> a = ra, b = rb, c = rc;
            if (MODE == 1 || MODE == 3) {
                a = sa[k];
                if (MODE == 1) {
                    b = sb[k];
                    c = sc[k];
                }
            } else {
                a.x += 1e-7f * k;  // a different entry each time
            }
            for (int u = 0; u < IB; ++u) {
                if (MODE <= 1)
                    bhq::pc_quad<float, false>(a, b, c, xi[u], yi[u], zi[u], e2, ax[u], ay[u],
                                               az[u], pt[u]);
                else
                    bhq::pp_plummer<float>(a, xi[u], yi[u], zi[u], e2, ax[u], ay[u], az[u],
                                           pt[u]);
            }
        }
    }
    const unsigned long long c1 = __builtin_amdgcn_s_memtime();
    const unsigned long long r1 = __builtin_amdgcn_s_memrealtime();
    float s = 0;
    for (int u = 0; u < IB; ++u) s += ax[u] + ay[u] + az[u] + pt[u];
    out[blockIdx.x * 256 + t] = s;
    if ((t & 63) == 0) {
        const int w = blockIdx.x * 4 + t / 64;
        cyc[2 * w] = c1 - c0;
        cyc[2 * w + 1] = r1 - r0;
    }
}

template <int MODE, int IB>
void run(int bpc, int ncu, float *out, unsigned long long *cyc, const V4<float> *src, int iters)
{
    const int grid = bpc * ncu;
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    hipLaunchKernelGGL((body<MODE, IB>), dim3(grid), dim3(256), 0, 0, out, cyc, iters, src);
    CHECK(hipEventRecord(e0, 0));
    hipLaunchKernelGGL((body<MODE, IB>), dim3(grid), dim3(256), 0, 0, out, cyc, iters, src);
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
    const double inter = (double)grid * 256 * iters * 64 * IB;
    const double flops = inter * (MODE <= 1 ? 53.0 : 20.0);
    const double instr = inter * (MODE <= 1 ? 34.0 : 14.0) / 64.0;  // wave-level
    const double quads = 4.0 * ncu * (clk_ghz * 1e9 * ms * 1e-3) / 4.0;  // SIMD quad-cycles
    const char *name[] = {"cell term, registers", "cell term, LDS", "particle term, registers",
                          "particle term, LDS"};
    std::printf("%-24s IB=%d waves/SIMD %d: %.3f ms, %.1f Ginteractions/s, %.1f TFLOP/s "
                "(%.3f of 157.3), clock %.3f GHz, %.3f term instructions per SIMD quad-cycle\n",
                name[MODE], IB, bpc, ms, inter / ms * 1e-6, flops / ms * 1e-9,
                flops / ms * 1e-9 / 157.3, clk_ghz, instr / quads);
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
}

template <int MODE, int IB>
void sweep(int ncu, float *out, unsigned long long *cyc, const V4<float> *src)
{
    for (int w : {2, 4, 5, 6, 8}) run<MODE, IB>(w, ncu, out, cyc, src, 200);
}

int main()
{
    hipDeviceProp_t p;
    CHECK(hipGetDeviceProperties(&p, 0));
    const int ncu = p.multiProcessorCount;
    std::printf("device %s, %d CUs\n", p.gcnArchName, ncu);
    float *out;
    unsigned long long *cyc;
    V4<float> *src;
    CHECK(hipMalloc(&out, (size_t)8 * ncu * 256 * sizeof(float)));
    CHECK(hipMalloc(&cyc, (size_t)8 * ncu * 4 * 2 * sizeof(unsigned long long)));
    CHECK(hipMalloc(&src, 192 * sizeof(V4<float>)));
    std::vector<V4<float>> h(192);
    for (int i = 0; i < 192; ++i)
        h[i] = {0.3f + 0.001f * i, -0.2f + 0.002f * i, 0.5f - 0.001f * i, 0.01f};
    CHECK(hipMemcpy(src, h.data(), h.size() * sizeof(V4<float>), hipMemcpyHostToDevice));
    sweep<0, 2>(ncu, out, cyc, src);
    sweep<1, 2>(ncu, out, cyc, src);
    sweep<1, 1>(ncu, out, cyc, src);
    sweep<2, 2>(ncu, out, cyc, src);
    sweep<3, 2>(ncu, out, cyc, src);
    CHECK(hipFree(out));
    CHECK(hipFree(cyc));
    CHECK(hipFree(src));
    return 0;
}
