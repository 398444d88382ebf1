// bhq_pm.hip -- particle-mesh long-range force, the complement of the
// Gaussian-split short-range tree kernels (together: TreePM; the paper's
// TreePM context, Sec. 1).
//
// The short-range pair potential is -erfc(r / 2 r_s) / r, so the long-range
// part is -erf(r / 2 r_s) / r, whose Fourier transform is
// -4 pi exp(-k^2 r_s^2) / k^2.  In the periodic box of side L (mean density
// removed, G = 1) on an n^3 mesh of spacing h = L / n:
//   1. triangular-shaped-cloud (TSC) assignment of the masses (mesh points
//      at integer multiples of h): the particles are radix-sorted by their
//      nearest mesh point, and one thread per mesh point sums, in a fixed
//      order, the particles of the 27 cells around it (no atomics: the
//      result is the same bits every run);
//   2. forward real-to-complex FFT (hipFFT);
//   3. one thread per complex mode: phi(k) = G(k) rho(k) with
//      G = -4 pi exp(-k^2 r_s^2) / k^2 / W(k)^2, W = prod_a sinc(k_a h/2)^3
//      (TSC window, assignment and interpolation), G(0) = 0, and the three
//      components -i k_a phi(k) (zero on the Nyquist planes);
//   4. four inverse complex-to-real FFTs (potential and acceleration);
//   5. the four meshes are interleaved into one (a_x, a_y, a_z, phi) record
//      per mesh point, and one thread per particle, in the sorted order,
//      interpolates them with the same TSC weights and writes its result
//      at the particle's input position.
// All FP64.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>
#include <hipfft/hipfft.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <new>
#include <string>

#include "bhq.h"
#include "bhq_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr double kPi = 3.14159265358979323846;

inline unsigned nblocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

struct Tsc {
    int i[3];        // nearest mesh index per axis (already mod n)
    double w[3][3];  // weights for offsets -1, 0, +1 per axis
};

__device__ __forceinline__ Tsc tsc(const double *x, double ih, int n)
{
    Tsc t;
    for (int a = 0; a < 3; ++a) {
        const double u = x[a] * ih;
        const double i0 = floor(u + 0.5);
        const double d = u - i0;
        int64_t k = (int64_t)i0 % n;
        if (k < 0) k += n;
        t.i[a] = (int)k;
        t.w[0][a] = 0.5 * (0.5 - d) * (0.5 - d);
        t.w[1][a] = 0.75 - d * d;
        t.w[2][a] = 0.5 * (0.5 + d) * (0.5 + d);
    }
    return t;
}

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Cell of the nearest mesh point of each particle, and the identity order.
__global__ __launch_bounds__(kBlock) void k_cell_keys(int64_t np, const double *x, double ih,
                                                      int n, uint32_t *key, int32_t *idx)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= np) return;
    const Tsc t = tsc(x + 3 * p, ih, n);
    key[p] = (uint32_t)(((int64_t)t.i[0] * n + t.i[1]) * n + t.i[2]);
    idx[p] = (int32_t)p;
}

// Sorted particle records (x, y, z, m) and each cell's range [start, end).
__global__ __launch_bounds__(kBlock) void k_sorted(int64_t np, const uint32_t *key,
                                                   const int32_t *idx, const double *x,
                                                   const double *m, double4 *xs,
                                                   int32_t *start, int32_t *end)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= np) return;
    const int64_t p = idx[k];
    xs[k] = make_double4(x[3 * p], x[3 * p + 1], x[3 * p + 2], m[p]);
    const uint32_t c = key[k];
    if (k == 0 || key[k - 1] != c) start[c] = (int32_t)k;
    if (k == np - 1 || key[k + 1] != c) end[c] = (int32_t)(k + 1);
}

// rho at mesh point q: the particles whose nearest point is q - o,
// o in {-1, 0, 1}^3, each with its TSC weight for offset o.
__global__ __launch_bounds__(kBlock) void k_gather_rho(int n, double ih, const double4 *xs,
                                                       const int32_t *start,
                                                       const int32_t *end, double *rho)
{
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t n3 = (int64_t)n * n * n;
    if (q >= n3) return;
    const int qz = (int)(q % n), qy = (int)((q / n) % n), qx = (int)(q / ((int64_t)n * n));
    double sum = 0.0;
    for (int ox = -1; ox <= 1; ++ox) {
        const int cx = wrap(qx - ox, n);
        for (int oy = -1; oy <= 1; ++oy) {
            const int cy = wrap(qy - oy, n);
            for (int oz = -1; oz <= 1; ++oz) {
                const int cz = wrap(qz - oz, n);
                const int64_t c = ((int64_t)cx * n + cy) * n + cz;
                const int32_t e = end[c];
                for (int32_t k = start[c]; k < e; ++k) {
                    const double4 r = xs[k];
                    const double xp[3] = {r.x, r.y, r.z};
                    const Tsc t = tsc(xp, ih, n);
                    sum += r.w * t.w[ox + 1][0] * t.w[oy + 1][1] * t.w[oz + 1][2];
                }
            }
        }
    }
    rho[q] = sum;
}

__device__ __forceinline__ double sinc_half(double kh)
{
    // sin(kh/2) / (kh/2), 1 at k = 0
    const double t = 0.5 * kh;
    return t == 0.0 ? 1.0 : sin(t) / t;
}

// rk: n x n x (n/2+1) complex; writes phik and the three gradient arrays.
__global__ __launch_bounds__(kBlock) void k_green(const hipfftDoubleComplex *rk, int n,
                                                  double L, double rs, double scale,
                                                  hipfftDoubleComplex *phik,
                                                  hipfftDoubleComplex *axk,
                                                  hipfftDoubleComplex *ayk,
                                                  hipfftDoubleComplex *azk)
{
    const int nz = n / 2 + 1;
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= (int64_t)n * n * nz) return;
    const int iz = (int)(e % nz);
    const int iy = (int)((e / nz) % n);
    const int ix = (int)(e / ((int64_t)nz * n));
    const double dk = 2.0 * kPi / L, h = L / n;
    // signed frequencies: index i < n/2 is i, the rest i - n (n/2 is -n/2)
    const double kxs = dk * (ix < n / 2 ? ix : ix - n);
    const double kys = dk * (iy < n / 2 ? iy : iy - n);
    const double kz = dk * iz;
    const double k2 = kxs * kxs + kys * kys + kz * kz;
    double g = 0.0;
    if (k2 > 0.0) {
        const double w = sinc_half(kxs * h) * sinc_half(kys * h) * sinc_half(kz * h);
        const double w3 = w * w * w;
        g = -4.0 * kPi * exp(-k2 * rs * rs) / k2 / (w3 * w3) * scale;
    }
    const hipfftDoubleComplex r = rk[e];
    const double pr = g * r.x, pi = g * r.y;
    phik[e] = make_hipDoubleComplex(pr, pi);
    // -i k phi = (k phi_i, -k phi_r)
    const double gx = ix == n / 2 ? 0.0 : kxs;
    const double gy = iy == n / 2 ? 0.0 : kys;
    const double gz = iz == n / 2 ? 0.0 : kz;
    axk[e] = make_hipDoubleComplex(gx * pi, -gx * pr);
    ayk[e] = make_hipDoubleComplex(gy * pi, -gy * pr);
    azk[e] = make_hipDoubleComplex(gz * pi, -gz * pr);
}

__global__ __launch_bounds__(kBlock) void k_interleave(int64_t n3, const double *axm,
                                                       const double *aym, const double *azm,
                                                       const double *phim, double4 *m4)
{
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= n3) return;
    m4[q] = make_double4(axm[q], aym[q], azm[q], phim[q]);
}

// Particle k of the sorted order: 27-point TSC interpolation of the
// interleaved mesh; the result goes to the particle's input index.
__global__ __launch_bounds__(kBlock) void k_interp(int64_t np, const double4 *xs,
                                                   const int32_t *idx, double ih, int n,
                                                   const double4 *m4, double *a, double *pot,
                                                   int accumulate)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= np) return;
    const double4 r = xs[k];
    const double xp[3] = {r.x, r.y, r.z};
    const Tsc t = tsc(xp, ih, n);
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int a0 = 0; a0 < 3; ++a0) {
        const int ix = wrap(t.i[0] + a0 - 1, n);
        for (int b = 0; b < 3; ++b) {
            const int iy = wrap(t.i[1] + b - 1, n);
            for (int c = 0; c < 3; ++c) {
                const int iz = wrap(t.i[2] + c - 1, n);
                const double4 v = m4[((int64_t)ix * n + iy) * n + iz];
                const double w = t.w[a0][0] * t.w[b][1] * t.w[c][2];
                s[0] += w * v.x;
                s[1] += w * v.y;
                s[2] += w * v.z;
                s[3] += w * v.w;
            }
        }
    }
    const int64_t p = idx[k];
    if (accumulate) {
        a[3 * p] += s[0];
        a[3 * p + 1] += s[1];
        a[3 * p + 2] += s[2];
        if (pot) pot[p] += s[3];
    } else {
        a[3 * p] = s[0];
        a[3 * p + 1] = s[1];
        a[3 * p + 2] = s[2];
        if (pot) pot[p] = s[3];
    }
}

}  // namespace

struct bhq_pm {
    int device = 0;
    int n = 0;
    double box = 0.0, rs = 0.0;
    std::string err;
    bhq::DevArray rho, rk, phik, axk, ayk, azk, phim, axm, aym, azm, m4;
    // per-particle sorting (grown to the largest n seen)
    bhq::DevArray key, key2, idx, idx2, xs, sort_tmp, start, end;
    hipfftHandle fwd = 0, inv = 0;
    bool have_fwd = false, have_inv = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool launched = false;

    int fail(int code, const char *fmt, ...)
    {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        err = buf;
        return code;
    }
};

namespace {

thread_local std::string g_pm_create_error;

void pm_free(bhq_pm *p)
{
    if (p->have_fwd) (void)hipfftDestroy(p->fwd);
    if (p->have_inv) (void)hipfftDestroy(p->inv);
    for (bhq::DevArray *a : {&p->rho, &p->rk, &p->phik, &p->axk, &p->ayk, &p->azk, &p->phim,
                             &p->axm, &p->aym, &p->azm, &p->m4, &p->key, &p->key2, &p->idx,
                             &p->idx2, &p->xs, &p->sort_tmp, &p->start, &p->end})
        a->release();
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    delete p;
}

int check_range(bhq_pm *pm, const void *ptr, size_t bytes, const char *name)
{
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, const_cast<void *>(ptr)) != hipSuccess || !base) {
        (void)hipGetLastError();
        return pm->fail(BHQ_E_ARG, "%s is not device memory", name);
    }
    const char *b = static_cast<const char *>(base);
    const char *q = static_cast<const char *>(ptr);
    if (q < b || (size_t)(q - b) + bytes > size)
        return pm->fail(BHQ_E_RANGE, "%s: %zu bytes do not fit its allocation", name, bytes);
    return BHQ_OK;
}

}  // namespace

extern "C" {

int bhq_pm_create(bhq_pm **out, int device, int nmesh, double box, double rs)
{
    if (!out) return BHQ_E_ARG;
    *out = nullptr;
    if (nmesh < 4 || nmesh > 1024 || (nmesh & 1) || !(box > 0.0) || !std::isfinite(box) ||
        !(rs > 0.0) || !std::isfinite(rs)) {
        g_pm_create_error = "bhq_pm_create: need an even mesh size in [4, 1024], box > 0, rs > 0";
        return BHQ_E_ARG;
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        g_pm_create_error = "bhq_pm_create: no such device";
        return BHQ_E_NODEV;
    }
    if (hipSetDevice(device) != hipSuccess) {
        g_pm_create_error = "bhq_pm_create: hipSetDevice failed";
        return BHQ_E_HIP;
    }
    bhq_pm *p = new (std::nothrow) bhq_pm();
    if (!p) {
        g_pm_create_error = "bhq_pm_create: out of host memory";
        return BHQ_E_NOMEM;
    }
    p->device = device;
    p->n = nmesh;
    p->box = box;
    p->rs = rs;
    const size_t n3 = (size_t)nmesh * nmesh * nmesh;
    const size_t nc = (size_t)nmesh * nmesh * (nmesh / 2 + 1);
    hipError_t e = hipSuccess;
    for (bhq::DevArray *a : {&p->rho, &p->phim, &p->axm, &p->aym, &p->azm})
        if (e == hipSuccess) e = a->reserve(n3 * sizeof(double));
    for (bhq::DevArray *a : {&p->rk, &p->phik, &p->axk, &p->ayk, &p->azk})
        if (e == hipSuccess) e = a->reserve(nc * sizeof(hipfftDoubleComplex));
    if (e == hipSuccess) e = p->m4.reserve(n3 * sizeof(double4));
    if (e == hipSuccess) e = p->start.reserve(n3 * sizeof(int32_t));
    if (e == hipSuccess) e = p->end.reserve(n3 * sizeof(int32_t));
    if (e == hipSuccess) e = hipEventCreate(&p->ev0);
    if (e == hipSuccess) e = hipEventCreate(&p->ev1);
    if (e != hipSuccess) {
        g_pm_create_error = std::string("bhq_pm_create: ") + hipGetErrorString(e);
        const int code = (e == hipErrorOutOfMemory) ? BHQ_E_NOMEM : BHQ_E_HIP;
        pm_free(p);
        return code;
    }
    if (hipfftPlan3d(&p->fwd, nmesh, nmesh, nmesh, HIPFFT_D2Z) != HIPFFT_SUCCESS) {
        g_pm_create_error = "bhq_pm_create: hipFFT forward plan failed";
        pm_free(p);
        return BHQ_E_HIP;
    }
    p->have_fwd = true;
    if (hipfftPlan3d(&p->inv, nmesh, nmesh, nmesh, HIPFFT_Z2D) != HIPFFT_SUCCESS) {
        g_pm_create_error = "bhq_pm_create: hipFFT inverse plan failed";
        pm_free(p);
        return BHQ_E_HIP;
    }
    p->have_inv = true;
    g_pm_create_error.clear();
    *out = p;
    return BHQ_OK;
}

int bhq_pm_destroy(bhq_pm *pm)
{
    if (!pm) return BHQ_OK;
    (void)hipSetDevice(pm->device);
    if (pm->launched) (void)hipEventSynchronize(pm->ev1);
    pm_free(pm);
    return BHQ_OK;
}

int bhq_pm_compute(bhq_pm *pm, int64_t np, const double *x, const double *m, double *a,
                   double *pot, int accumulate, void *stream)
{
    if (!pm) return BHQ_E_ARG;
    if (np < 1 || np > 0x7fffffffLL || !x || !m || !a || (accumulate != 0 && accumulate != 1))
        return pm->fail(BHQ_E_ARG, "pm_compute: bad argument");
    if (hipSetDevice(pm->device) != hipSuccess) return pm->fail(BHQ_E_HIP, "hipSetDevice");
    int rc = check_range(pm, x, (size_t)np * 3 * sizeof(double), "x");
    if (rc == BHQ_OK) rc = check_range(pm, m, (size_t)np * sizeof(double), "m");
    if (rc == BHQ_OK) rc = check_range(pm, a, (size_t)np * 3 * sizeof(double), "a");
    if (rc == BHQ_OK && pot) rc = check_range(pm, pot, (size_t)np * sizeof(double), "pot");
    if (rc != BHQ_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int n = pm->n;
    const double h = pm->box / n, ih = 1.0 / h;
    const size_t n3 = (size_t)n * n * n;
    const int64_t nc = (int64_t)n * n * (n / 2 + 1);
    // density = mass / h^3; the inverse transforms are unnormalised (1/n^3)
    const double scale = 1.0 / (h * h * h) / (double)n3;
    auto hipok = [&](hipError_t e, const char *w) -> bool {
        if (e == hipSuccess) return true;
        pm->fail(BHQ_E_HIP, "pm_compute: %s: %s", w, hipGetErrorString(e));
        return false;
    };
    auto fftok = [&](hipfftResult r, const char *w) -> bool {
        if (r == HIPFFT_SUCCESS) return true;
        pm->fail(BHQ_E_HIP, "pm_compute: %s failed (hipFFT %d)", w, (int)r);
        return false;
    };
    if (!hipok(hipEventRecord(pm->ev0, s), "event")) return BHQ_E_HIP;
    // particles sorted by their nearest mesh point, cell ranges, density
    for (bhq::DevArray *b : {&pm->key, &pm->key2})
        if (!hipok(b->reserve((size_t)np * 4), "allocation")) return BHQ_E_NOMEM;
    for (bhq::DevArray *b : {&pm->idx, &pm->idx2})
        if (!hipok(b->reserve((size_t)np * 4), "allocation")) return BHQ_E_NOMEM;
    if (!hipok(pm->xs.reserve((size_t)np * sizeof(double4)), "allocation")) return BHQ_E_NOMEM;
    int bits = 1;
    while (((uint64_t)1 << bits) < (uint64_t)n3) ++bits;
    size_t tmp = 0;
    if (!hipok(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, pm->key.as<uint32_t>(),
                                                  pm->key2.as<uint32_t>(), pm->idx.as<int32_t>(),
                                                  pm->idx2.as<int32_t>(), (int)np, 0, bits, s),
               "sort size"))
        return BHQ_E_HIP;
    if (!hipok(pm->sort_tmp.reserve(tmp), "allocation")) return BHQ_E_NOMEM;
    hipLaunchKernelGGL(k_cell_keys, dim3(nblocks(np)), dim3(kBlock), 0, s, np, x, ih, n,
                       pm->key.as<uint32_t>(), pm->idx.as<int32_t>());
    if (!hipok(hipGetLastError(), "cell keys")) return BHQ_E_HIP;
    if (!hipok(hipcub::DeviceRadixSort::SortPairs(pm->sort_tmp.p, tmp, pm->key.as<uint32_t>(),
                                                  pm->key2.as<uint32_t>(), pm->idx.as<int32_t>(),
                                                  pm->idx2.as<int32_t>(), (int)np, 0, bits, s),
               "sort"))
        return BHQ_E_HIP;
    if (!hipok(hipMemsetAsync(pm->start.p, 0, n3 * sizeof(int32_t), s), "memset") ||
        !hipok(hipMemsetAsync(pm->end.p, 0, n3 * sizeof(int32_t), s), "memset"))
        return BHQ_E_HIP;
    hipLaunchKernelGGL(k_sorted, dim3(nblocks(np)), dim3(kBlock), 0, s, np,
                       pm->key2.as<uint32_t>(), pm->idx2.as<int32_t>(), x, m,
                       pm->xs.as<double4>(), pm->start.as<int32_t>(), pm->end.as<int32_t>());
    if (!hipok(hipGetLastError(), "sorted records")) return BHQ_E_HIP;
    hipLaunchKernelGGL(k_gather_rho, dim3(nblocks((int64_t)n3)), dim3(kBlock), 0, s, n, ih,
                       pm->xs.as<double4>(), pm->start.as<int32_t>(), pm->end.as<int32_t>(),
                       pm->rho.as<double>());
    if (!hipok(hipGetLastError(), "assignment")) return BHQ_E_HIP;
    if (!fftok(hipfftSetStream(pm->fwd, s), "set stream") ||
        !fftok(hipfftSetStream(pm->inv, s), "set stream"))
        return BHQ_E_HIP;
    if (!fftok(hipfftExecD2Z(pm->fwd, pm->rho.as<hipfftDoubleReal>(),
                             pm->rk.as<hipfftDoubleComplex>()),
               "forward FFT"))
        return BHQ_E_HIP;
    hipLaunchKernelGGL(k_green, dim3(nblocks(nc)), dim3(kBlock), 0, s,
                       pm->rk.as<hipfftDoubleComplex>(), n, pm->box, pm->rs, scale,
                       pm->phik.as<hipfftDoubleComplex>(), pm->axk.as<hipfftDoubleComplex>(),
                       pm->ayk.as<hipfftDoubleComplex>(), pm->azk.as<hipfftDoubleComplex>());
    if (!hipok(hipGetLastError(), "green function")) return BHQ_E_HIP;
    const struct { bhq::DevArray *in, *out; } inv[] = {
        {&pm->phik, &pm->phim}, {&pm->axk, &pm->axm}, {&pm->ayk, &pm->aym}, {&pm->azk, &pm->azm}};
    for (auto &t : inv)
        if (!fftok(hipfftExecZ2D(pm->inv, t.in->as<hipfftDoubleComplex>(),
                                 t.out->as<hipfftDoubleReal>()),
                   "inverse FFT"))
            return BHQ_E_HIP;
    hipLaunchKernelGGL(k_interleave, dim3(nblocks((int64_t)n3)), dim3(kBlock), 0, s,
                       (int64_t)n3, pm->axm.as<double>(), pm->aym.as<double>(),
                       pm->azm.as<double>(), pm->phim.as<double>(), pm->m4.as<double4>());
    if (!hipok(hipGetLastError(), "interleave")) return BHQ_E_HIP;
    hipLaunchKernelGGL(k_interp, dim3(nblocks(np)), dim3(kBlock), 0, s, np,
                       pm->xs.as<double4>(), pm->idx2.as<int32_t>(), ih, n,
                       pm->m4.as<double4>(), a, pot, accumulate);
    if (!hipok(hipGetLastError(), "interpolation")) return BHQ_E_HIP;
    if (!hipok(hipEventRecord(pm->ev1, s), "event")) return BHQ_E_HIP;
    pm->launched = true;
    return BHQ_OK;
}

int bhq_pm_get_ms(bhq_pm *pm, double *ms)
{
    if (!pm || !ms) return BHQ_E_ARG;
    if (!pm->launched) return pm->fail(BHQ_E_STATE, "pm_get_ms before compute");
    float f = 0.0f;
    if (hipEventSynchronize(pm->ev1) != hipSuccess ||
        hipEventElapsedTime(&f, pm->ev0, pm->ev1) != hipSuccess)
        return pm->fail(BHQ_E_HIP, "pm_get_ms: event query failed");
    *ms = f;
    return BHQ_OK;
}

const char *bhq_pm_last_error(const bhq_pm *pm)
{
    return pm ? pm->err.c_str() : g_pm_create_error.c_str();
}

}  // extern "C"
