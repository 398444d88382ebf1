// bhq_integrate.hip -- what a time step needs around the force evaluation:
// results back in the particles' input order, the leapfrog kick and drift,
// and the kinetic and potential energies.  All arrays are FP64 in device
// memory.
#include <hip/hip_runtime.h>

#include "bhq.h"
#include "bhq_internal.h"

namespace bhq {

namespace {

constexpr int kBlock = 256;
constexpr int kEnergyBlocks = 512;

inline unsigned blocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// a_in[k] (group order) -> a_out[order[k]] (input order).
__global__ __launch_bounds__(kBlock) void k_scatter(const int32_t *order, int64_t n,
                                                    const double *ax, const double *ay,
                                                    const double *az, const double *pot,
                                                    double *a_out, double *pot_out)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const int64_t p = order ? order[k] : k;
    a_out[3 * p] = ax[k];
    a_out[3 * p + 1] = ay[k];
    a_out[3 * p + 2] = az[k];
    if (pot_out) pot_out[p] = pot[k];
}

// v += dtk a, then x += dtd v.
__global__ __launch_bounds__(kBlock) void k_kick_drift(int64_t n, double *x, double *v,
                                                       const double *a, double dtk,
                                                       double dtd)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= 3 * n) return;
    const double vn = v[i] + dtk * a[i];
    v[i] = vn;
    if (dtd != 0.0) x[i] = x[i] + dtd * vn;
}

// x <- x - box floor(x / box), then one more box off if rounding left it
// at box: the periodic image in [0, box).
__global__ __launch_bounds__(kBlock) void k_wrap(int64_t n3, double *x, double box)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n3) return;
    double y = x[i] - box * floor(x[i] / box);
    if (y >= box) y -= box;
    x[i] = y;
}

// out row k = in row order[k], rows of w 8-byte words.
__global__ __launch_bounds__(kBlock) void k_gather_rows(int64_t n, int w, const uint64_t *in,
                                                        const int32_t *order, uint64_t *out)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n * w) return;
    const int64_t k = i / w;
    const int c = (int)(i - k * w);
    out[i] = in[(int64_t)order[k] * w + c];
}

__global__ __launch_bounds__(kBlock) void k_iota(int32_t *v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) v[i] = (int32_t)i;
}

__global__ __launch_bounds__(kBlock) void k_fill_f64(double *v, int64_t n, double val)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) v[i] = val;
}

// Per-block partial sums of K = 1/2 sum m |v|^2 and
// W = 1/2 sum m (phi + m / eps) (the self pair's -m/eps removed), each
// block over a fixed strided range, combined in a fixed order: the result
// does not depend on scheduling.
__global__ __launch_bounds__(kBlock) void k_energy_partial(int64_t n, const double *m,
                                                           const double *v,
                                                           const double *pot, double eps,
                                                           double *part)
{
    __shared__ double sk[kBlock], sw[kBlock];
    double k = 0.0, w = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const double vx = v[3 * i], vy = v[3 * i + 1], vz = v[3 * i + 2];
        k += m[i] * (vx * vx + vy * vy + vz * vz);
        if (pot) w += m[i] * (pot[i] + (eps > 0.0 ? m[i] / eps : 0.0));
    }
    sk[threadIdx.x] = k;
    sw[threadIdx.x] = w;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sk[threadIdx.x] += sk[threadIdx.x + h];
            sw[threadIdx.x] += sw[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = 0.5 * sk[0];
        part[2 * blockIdx.x + 1] = 0.5 * sw[0];
    }
}

__global__ __launch_bounds__(kBlock) void k_energy_final(const double *part, int nb,
                                                         double *out)
{
    __shared__ double sk[kBlock], sw[kBlock];
    double k = 0.0, w = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) {
        k += part[2 * b];
        w += part[2 * b + 1];
    }
    sk[threadIdx.x] = k;
    sw[threadIdx.x] = w;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sk[threadIdx.x] += sk[threadIdx.x + h];
            sw[threadIdx.x] += sw[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sk[0];
        out[1] = sw[0];
    }
}

}  // namespace

hipError_t launch_scatter(const int32_t *order, int64_t n, const double *ax,
                          const double *ay, const double *az, const double *pot,
                          double *a_out, double *pot_out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3(blocks(n)), dim3(kBlock), 0, s, order, n, ax, ay, az,
                       pot, a_out, pot_out);
    return hipGetLastError();
}

hipError_t launch_kick_drift(int64_t n, double *x, double *v, const double *a, double dtk,
                             double dtd, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_kick_drift, dim3(blocks(3 * n)), dim3(kBlock), 0, s, n, x, v, a, dtk,
                       dtd);
    return hipGetLastError();
}

hipError_t launch_wrap(int64_t n, double *x, double box, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_wrap, dim3(blocks(3 * n)), dim3(kBlock), 0, s, 3 * n, x, box);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *v, int64_t n, double val, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64, dim3(blocks(n)), dim3(kBlock), 0, s, v, n, val);
    return hipGetLastError();
}

hipError_t launch_gather_rows(int64_t n, int words, const void *in, const int32_t *order,
                              void *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_rows, dim3(blocks(n * words)), dim3(kBlock), 0, s, n, words,
                       static_cast<const uint64_t *>(in), order, static_cast<uint64_t *>(out));
    return hipGetLastError();
}

hipError_t launch_iota(int32_t *v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_iota, dim3(blocks(n)), dim3(kBlock), 0, s, v, n);
    return hipGetLastError();
}

int energy_partials() { return kEnergyBlocks; }

hipError_t launch_energies(int64_t n, const double *m, const double *v, const double *pot,
                           double eps, double *part, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_energy_partial, dim3(kEnergyBlocks), dim3(kBlock), 0, s, n, m, v, pot,
                       eps, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kBlock), 0, s, part, kEnergyBlocks, out);
    return hipGetLastError();
}

}  // namespace bhq
