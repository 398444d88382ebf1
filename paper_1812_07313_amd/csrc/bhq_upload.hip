// bhq_upload.hip -- device-side uploads for the set calls that read caller
// device memory (bhq_set_*_dev): validation of the caller's arrays into a
// flag word, and their copy into the context's layout (AoS columns to SoA
// arrays, pool records).  Every kernel only reads its inputs and writes the
// context's arrays; nothing is decided here that the host calls decide
// differently.
#include <hip/hip_runtime.h>

#include <cmath>

#include "bhq_internal.h"

namespace bhq {

namespace {

constexpr int kBlock = 256;

inline unsigned grid(int64_t n)
{
    const int64_t b = (n + kBlock - 1) / kBlock;
    return (unsigned)(b < 65535 * 16 ? (b > 0 ? b : 1) : 65535 * 16);
}

__global__ __launch_bounds__(kBlock) void k_clear(unsigned *flag)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 0u;
}

__global__ __launch_bounds__(kBlock) void k_check_f64(const double *v, int64_t n, int positive,
                                                      unsigned *flag)
{
    unsigned bad = 0;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * kBlock) {
        const double x = v[k];
        if (!isfinite(x)) bad |= kBadNonFinite;
        else if (positive && !(x >= kMinEps2)) bad |= kBadNonPositive;
    }
    if (bad) atomicOr(flag, bad);
}

// off[0] == 0 and off[g] <= off[g + 1] for g < ng
__global__ __launch_bounds__(kBlock) void k_check_offsets(const int64_t *off, int64_t ng,
                                                          unsigned *flag)
{
    unsigned bad = 0;
    for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < ng;
         g += (int64_t)gridDim.x * kBlock) {
        if (off[g + 1] < off[g]) bad |= kBadOrder;
        if (g == 0 && off[0] != 0) bad |= kBadOrder;
    }
    if (bad) atomicOr(flag, bad);
}

__global__ __launch_bounds__(kBlock) void k_check_idx(const int32_t *idx, int64_t n, int64_t pool,
                                                      unsigned *flag)
{
    unsigned bad = 0;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * kBlock) {
        const int32_t v = idx[k];
        if (v < 0 || (int64_t)v >= pool) bad |= kBadRange;
    }
    if (bad) atomicOr(flag, bad);
}

struct Cols {
    double *c[6];
};

// column c of the AoS array v[n][w] to out.c[c] (skipped where NULL)
__global__ __launch_bounds__(kBlock) void k_unpack(const double *v, int64_t n, int w, Cols out)
{
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * kBlock)
        for (int c = 0; c < w; ++c)
            if (out.c[c]) out.c[c][k] = v[k * w + c];
}

__global__ __launch_bounds__(kBlock) void k_pack_particles(const double *x, const double *m,
                                                           int64_t n, PartRec *out)
{
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * kBlock)
        out[k] = PartRec{x[3 * k], x[3 * k + 1], x[3 * k + 2], m[k]};
}

__global__ __launch_bounds__(kBlock) void k_pack_cells(const double *x, const double *m,
                                                       const double *q, const double *t,
                                                       int64_t n, CellRec *out)
{
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * kBlock) {
        const double *qk = q + 6 * k;
        out[k] = CellRec{x[3 * k], x[3 * k + 1], x[3 * k + 2], m[k], qk[0], qk[1], qk[2],
                         qk[3], qk[4], qk[5], t ? t[k] : 0.0, 0.0};
    }
}

}  // namespace

hipError_t launch_clear_flag(unsigned *flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear, dim3(1), dim3(kBlock), 0, s, flag);
    return hipGetLastError();
}

hipError_t launch_check_f64(const double *v, int64_t n, bool positive, unsigned *flag,
                            hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_f64, dim3(grid(n)), dim3(kBlock), 0, s, v, n, positive ? 1 : 0,
                       flag);
    return hipGetLastError();
}

hipError_t launch_check_offsets(const int64_t *off, int64_t ng, unsigned *flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_offsets, dim3(grid(ng)), dim3(kBlock), 0, s, off, ng, flag);
    return hipGetLastError();
}

hipError_t launch_check_idx(const int32_t *idx, int64_t n, int64_t pool, unsigned *flag,
                            hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_idx, dim3(grid(n)), dim3(kBlock), 0, s, idx, n, pool, flag);
    return hipGetLastError();
}

hipError_t launch_unpack(const double *v, int64_t n, int w, double *const *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (w < 1 || w > 6) return hipErrorInvalidValue;
    Cols c{};
    for (int k = 0; k < w; ++k) c.c[k] = out[k];
    hipLaunchKernelGGL(k_unpack, dim3(grid(n)), dim3(kBlock), 0, s, v, n, w, c);
    return hipGetLastError();
}

hipError_t launch_pack_particles(const double *x, const double *m, int64_t n, PartRec *out,
                                 hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_particles, dim3(grid(n)), dim3(kBlock), 0, s, x, m, n, out);
    return hipGetLastError();
}

hipError_t launch_pack_cells(const double *x, const double *m, const double *q,
                             const double *t, int64_t n, CellRec *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_cells, dim3(grid(n)), dim3(kBlock), 0, s, x, m, q, t, n, out);
    return hipGetLastError();
}

}  // namespace bhq
