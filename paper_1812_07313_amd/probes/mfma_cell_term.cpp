// mfma_cell_term -- can the matrix cores take part of the quadrupole cell
// term?  For the pairs (i, c) of a group, the products Q_c d with
// d = x_c - x_i form a matrix product with inner dimension 4:
//   (Q_c d)[m] = sum_k A[(c, m)][k] B[k][i],
//   A[(c, m)][k] = -Q_c[m][k] (k < 3),  A[(c, m)][3] = (Q_c x_c)[m],
//   B[k][i] = x_i[k] (k < 3),  B[3][i] = 1.
// One v_mfma_f32_16x16x4f32 then covers 4 cells (rows 4c + m, m = 3 a zero
// row) and 16 i-particles, and lane l receives the whole Q d of pair
// (i = l % 16, cell l / 16).  The program first checks that lane layout on
// one wave (lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and
// holds D[4 (l / 16) + v][l % 16]), then times the cell term in that form
// (Q d from the matrix core, the other 25 operations on the VALU, one pair
// per lane per step) against the force kernels' VALU term (bhq_terms.h,
// two i-particles per lane, entries as LDS broadcasts), at 4, 5, 6 and 8
// waves per SIMD, with the clock the waves measured.
//
//   mfma_cell_term
#include <hip/hip_runtime.h>

#include <cmath>
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
typedef float v4f __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(64) void layout(const float *a, const float *b, float *d)
{
    const int l = threadIdx.x;
    const v4f zero = {0.f, 0.f, 0.f, 0.f};
    const v4f r = __builtin_amdgcn_mfma_f32_16x16x4f32(a[l], b[l], zero, 0, 0, 0);
    for (int v = 0; v < 4; ++v) d[l * 4 + v] = r[v];
}

// MODE 0: the VALU cell term, two i-particles per lane, 64 entries from LDS
// MODE 1: Q d from the matrix core, 16 steps of 4 cells per pass
template <int MODE>
__global__ __launch_bounds__(256) void body(float *out, unsigned long long *cyc, int iters,
                                            const V4<float> *src, const float *srcA)
{
    __shared__ V4<float> sa[64], sb[64], sc[64];
    __shared__ float sA[16 * 64];
    const int t = threadIdx.x;
    if (t < 64) {
        sa[t] = src[t];
        sb[t] = src[64 + t];
        sc[t] = src[128 + t];
    }
    for (int k = t; k < 16 * 64; k += 256) sA[k] = srcA[k];
    __syncthreads();
    const float e2 = 1e-4f;
    float s = 0.0f;
    const unsigned long long c0 = __builtin_amdgcn_s_memtime();
    const unsigned long long r0 = __builtin_amdgcn_s_memrealtime();
    if constexpr (MODE == 0) {
        float xi[2], yi[2], zi[2], ax[2], ay[2], az[2], pt[2];
        for (int u = 0; u < 2; ++u) {
            xi[u] = 0.01f * (t + u);
            yi[u] = 0.02f * u;
            zi[u] = -0.01f * t;
            ax[u] = ay[u] = az[u] = pt[u] = 0.0f;
        }
        for (int it = 0; it < iters; ++it) {
#pragma unroll 2
            for (int k = 0; k < 64; ++k) {
                const V4<float> a = sa[k], b = sb[k], c = sc[k];
                for (int u = 0; u < 2; ++u)
                    bhq::pc_quad<float, false>(a, b, c, xi[u], yi[u], zi[u], e2, ax[u], ay[u],
                                               az[u], pt[u]);
            }
        }
        for (int u = 0; u < 2; ++u) s += ax[u] + ay[u] + az[u] + pt[u];
    } else {
        const int l = t & 63;
        const int kk = l >> 4;  // the lane's cell within a step, and its k for B
        const float xi = 0.01f * (l & 15), yi = 0.02f * (t >> 6), zi = -0.01f * (l & 15);
        const float bop = kk == 0 ? xi : kk == 1 ? yi : kk == 2 ? zi : 1.0f;
        float ax = 0.f, ay = 0.f, az = 0.f, pt = 0.f;
        const v4f zero = {0.f, 0.f, 0.f, 0.f};
        for (int it = 0; it < iters; ++it) {
#pragma unroll 8
            for (int g = 0; g < 16; ++g) {
                const v4f q = __builtin_amdgcn_mfma_f32_16x16x4f32(sA[g * 64 + l], bop, zero, 0,
                                                                   0, 0);
                const V4<float> rec = sa[g * 4 + kk];
                const float dx = rec.x - xi, dy = rec.y - yi, dz = rec.z - zi;
                const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, e2)));
                const float rinv = bhq::rsq(r2);
                const float rinv2 = rinv * rinv;
                const float phim = rec.w * rinv;
                const float dqd = fmaf(dz, q[2], fmaf(dy, q[1], dx * q[0]));
                const float rinv5 = (rinv2 * rinv2) * rinv;
                const float pq = dqd * rinv5;
                pt += phim;
                pt = fmaf(0.5f, pq, pt);
                const float cf = fmaf(2.5f, pq, phim) * rinv2;
                ax = fmaf(cf, dx, ax);
                ay = fmaf(cf, dy, ay);
                az = fmaf(cf, dz, az);
                ax = fmaf(-rinv5, q[0], ax);
                ay = fmaf(-rinv5, q[1], ay);
                az = fmaf(-rinv5, q[2], az);
            }
        }
        s = ax + ay + az + pt;
    }
    const unsigned long long c1 = __builtin_amdgcn_s_memtime();
    const unsigned long long r1 = __builtin_amdgcn_s_memrealtime();
    out[blockIdx.x * 256 + t] = s;
    if ((t & 63) == 0) {
        const int w = blockIdx.x * 4 + t / 64;
        cyc[2 * w] = c1 - c0;
        cyc[2 * w + 1] = r1 - r0;
    }
}

template <int MODE>
void run(int bpc, int ncu, float *out, unsigned long long *cyc, const V4<float> *src,
         const float *srcA, int iters)
{
    const int grid = bpc * ncu;
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    hipLaunchKernelGGL((body<MODE>), dim3(grid), dim3(256), 0, 0, out, cyc, iters, src, srcA);
    CHECK(hipEventRecord(e0, 0));
    hipLaunchKernelGGL((body<MODE>), dim3(grid), dim3(256), 0, 0, out, cyc, iters, src, srcA);
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
    const double clk = cs / (rs * 10.0);  // s_memrealtime counts at 100 MHz
    // pairs: MODE 0 64 entries x 2 i-particles per thread and pass; MODE 1
    // 16 steps x 1 pair per lane and pass
    const double pairs = (double)grid * 256 * iters * (MODE == 0 ? 128.0 : 16.0);
    std::printf("%s waves/SIMD %d: %.3f ms, %.1f G pairs/s, clock %.3f GHz, %.1f G pairs/s "
                "scaled to 2.2 GHz\n",
                MODE == 0 ? "VALU term, 2 i/lane     " : "MFMA Q d + VALU, 1 pair", bpc, ms,
                pairs / ms * 1e-6, clk, pairs / ms * 1e-6 * 2.2 / clk);
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
}

int main()
{
    hipDeviceProp_t p;
    CHECK(hipGetDeviceProperties(&p, 0));
    const int ncu = p.multiProcessorCount;
    std::printf("device %s, %d CUs\n", p.gcnArchName, ncu);

    // the lane layout, on one wave
    std::vector<float> ha(64), hb(64), hd(256);
    for (int l = 0; l < 64; ++l) {
        ha[l] = 1.0f + 0.5f * l;
        hb[l] = 2.0f - 0.25f * l;
    }
    float *da, *db, *dd;
    CHECK(hipMalloc(&da, 64 * sizeof(float)));
    CHECK(hipMalloc(&db, 64 * sizeof(float)));
    CHECK(hipMalloc(&dd, 256 * sizeof(float)));
    CHECK(hipMemcpy(da, ha.data(), 64 * sizeof(float), hipMemcpyHostToDevice));
    CHECK(hipMemcpy(db, hb.data(), 64 * sizeof(float), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(layout, dim3(1), dim3(64), 0, 0, da, db, dd);
    CHECK(hipDeviceSynchronize());
    CHECK(hipMemcpy(hd.data(), dd, 256 * sizeof(float), hipMemcpyDeviceToHost));
    double worst = 0;
    for (int l = 0; l < 64; ++l)
        for (int v = 0; v < 4; ++v) {
            const int i = 4 * (l / 16) + v, j = l % 16;
            double sum = 0;
            for (int k = 0; k < 4; ++k) sum += (double)ha[16 * k + i] * hb[16 * k + j];
            worst = std::fmax(worst, std::fabs(sum - hd[l * 4 + v]));
        }
    std::printf("16x16x4 f32 lane layout: max |D - A B| = %g (%s)\n", worst,
                worst < 1e-3 ? "as stated" : "DIFFERENT");
    CHECK(hipFree(da));
    CHECK(hipFree(db));
    CHECK(hipFree(dd));

    float *out, *srcA;
    unsigned long long *cyc;
    V4<float> *src;
    CHECK(hipMalloc(&out, (size_t)8 * ncu * 256 * sizeof(float)));
    CHECK(hipMalloc(&cyc, (size_t)8 * ncu * 4 * 2 * sizeof(unsigned long long)));
    CHECK(hipMalloc(&src, 192 * sizeof(V4<float>)));
    CHECK(hipMalloc(&srcA, 16 * 64 * sizeof(float)));
    std::vector<V4<float>> h(192);
    for (int i = 0; i < 192; ++i)
        h[i] = {0.3f + 0.001f * i, -0.2f + 0.002f * i, 0.5f - 0.001f * i, 0.01f};
    std::vector<float> hA(16 * 64);
    for (int i = 0; i < 16 * 64; ++i) hA[i] = 1e-3f * (float)((i * 37) % 17 - 8);
    CHECK(hipMemcpy(src, h.data(), h.size() * sizeof(V4<float>), hipMemcpyHostToDevice));
    CHECK(hipMemcpy(srcA, hA.data(), hA.size() * sizeof(float), hipMemcpyHostToDevice));
    for (int w : {4, 5, 6, 8}) {
        run<0>(w, ncu, out, cyc, src, srcA, 200);
        run<1>(w, ncu, out, cyc, src, srcA, 800);
    }
    CHECK(hipFree(out));
    CHECK(hipFree(cyc));
    CHECK(hipFree(src));
    CHECK(hipFree(srcA));
    return 0;
}
