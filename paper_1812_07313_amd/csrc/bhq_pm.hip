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
//      result is the same bits every run).  A block takes a tile of
//      2 x 8 x 16 mesh points and first copies the particles of the tile's
//      cells and their neighbours (720 cells) to LDS, so that each particle
//      is read from memory about twice instead of 27 times;
//   2. forward real-to-complex FFT (hipFFT);
//   3. one thread per complex mode: phi(k) = G(k) rho(k) with
//      G = -4 pi exp(-k^2 r_s^2) / k^2 / W(k)^2, W = prod_a sinc(k_a h/2)^3
//      (TSC window, assignment and interpolation), G(0) = 0, and the three
//      components -i k_a phi(k) (zero on the Nyquist planes);
//   4. four inverse complex-to-real FFTs (potential and acceleration);
//   5. the four meshes are interleaved into one (a_x, a_y, a_z, phi) record
//      per mesh point, and one thread per particle, in the sorted order,
//      interpolates them with the same TSC weights and writes its result
//      at the particle's input position.  A block takes the particles of a
//      tile of 2 x 8 x 16 cells, with the records of the tile's mesh points
//      and their neighbours in LDS.
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

// No contraction into fused multiply-adds: every kernel that locates a
// particle's mesh cell must get the bits the sort keys were made with.
#pragma clang fp contract(off)

namespace {

constexpr int kBlock = 256;
constexpr double kPi = 3.14159265358979323846;

inline unsigned nblocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

struct Tsc {
    int i[3];        // nearest mesh index per axis (already mod n)
    double w[3][3];  // weights for offsets -1, 0, +1 per axis
};

// Offset of coordinate x from its nearest mesh point, in mesh spacings.
__device__ __forceinline__ double tsc_d(double x, double ih, double &i0)
{
    const double u = x * ih;
    i0 = floor(u + 0.5);
    return u - i0;
}

// TSC weight of the mesh point at offset o (-1, 0, +1) for offset d.
__device__ __forceinline__ double tsc_w(double d, int o)
{
    return o < 0 ? 0.5 * (0.5 - d) * (0.5 - d)
                 : (o == 0 ? 0.75 - d * d : 0.5 * (0.5 + d) * (0.5 + d));
}

__device__ __forceinline__ Tsc tsc(const double *x, double ih, int n)
{
    Tsc t;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double i0;
        const double d = tsc_d(x[a], ih, i0);
        // i0 mod n; positions inside the box need no division
        int64_t k = (int64_t)i0;
        if (k < 0 || k >= n) {
            k %= n;
            if (k < 0) k += n;
        }
        t.i[a] = (int)k;
        t.w[0][a] = tsc_w(d, -1);
        t.w[1][a] = tsc_w(d, 0);
        t.w[2][a] = tsc_w(d, 1);
    }
    return t;
}

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// i mod n in [0, n) for any i (meshes smaller than a tile wrap several times)
__device__ __forceinline__ int pmod(int i, int n)
{
    const int r = i % n;
    return r < 0 ? r + n : r;
}

// Tiles of the mesh (points for the assignment, cells for the
// interpolation): kTX x kTY x kTZ per block of kBlock threads, z fastest;
// with their neighbours, kHX x kHY x kHZ.
constexpr int kTX = 2, kTY = 8, kTZ = 16;
constexpr int kHX = kTX + 2, kHY = kTY + 2, kHZ = kTZ + 2;
constexpr int kHalo = kHX * kHY * kHZ;
constexpr int kGatherCap = 896;  // particles of a tile's neighbourhood held in LDS
static_assert(kTX * kTY * kTZ == kBlock, "one tile point per thread");

inline unsigned ntiles(int n)
{
    return (unsigned)(((n + kTX - 1) / kTX) * ((n + kTY - 1) / kTY) * ((n + kTZ - 1) / kTZ));
}

// Origin of block b's tile.
__device__ __forceinline__ void tile_origin(int n, int &x0, int &y0, int &z0)
{
    const int nz = (n + kTZ - 1) / kTZ, ny = (n + kTY - 1) / kTY;
    int b = (int)blockIdx.x;
    z0 = (b % nz) * kTZ;
    b /= nz;
    y0 = (b % ny) * kTY;
    x0 = (b / ny) * kTX;
}

// Mesh index of neighbourhood entry h of the tile at (x0, y0, z0).
__device__ __forceinline__ int64_t halo_point(int h, int n, int x0, int y0, int z0)
{
    const int hz = h % kHZ, hy = (h / kHZ) % kHY, hx = h / (kHZ * kHY);
    const int cx = pmod(x0 - 1 + hx, n), cy = pmod(y0 - 1 + hy, n), cz = pmod(z0 - 1 + hz, n);
    return ((int64_t)cx * n + cy) * n + cz;
}

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

// TSC weight for offset o (-1, 0, +1) with o known only at run time; the
// same operations as tsc_w (negating d is exact).
__device__ __forceinline__ double tsc_w_var(double d, int o)
{
    const double s = o < 0 ? -d : d;
    return o == 0 ? 0.75 - d * d : 0.5 * (0.5 + s) * (0.5 + s);
}

// Sum over the neighbourhood of tile point (tx, ty, tz), row by row: for
// each (ox, oy) the cells at z offsets +1, 0, -1 (neighbourhood z indices
// tz .. tz + 2), each cell's particles in the sorted order.
// LDS: the three cells' particles are contiguous in sp, as (offsets from
// the nearest mesh point, m), with their neighbourhood z index in sz, so
// that a row is one loop.  Memory: cell by cell from xs, the same order.
__device__ __forceinline__ void gather_point_lds(int tx, int ty, int tz, const double4 *sp,
                                                 const uint8_t *sz, const int32_t *first,
                                                 const int32_t *count, double &sum)
{
#pragma unroll
    for (int ox = -1; ox <= 1; ++ox) {
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy) {
            const int h0 = ((tx + 1 - ox) * kHY + (ty + 1 - oy)) * kHZ + tz;
            const int32_t k0 = first[h0], k1 = first[h0 + 2] + count[h0 + 2];
            for (int32_t k = k0; k < k1; ++k) {
                const double4 r = sp[k];
                const int oz = tz + 1 - sz[k];
                sum += r.w * tsc_w(r.x, ox) * tsc_w(r.y, oy) * tsc_w_var(r.z, oz);
            }
        }
    }
}

__device__ __forceinline__ void gather_point_mem(int tx, int ty, int tz, double ih,
                                                 const double4 *xs, const int32_t *start,
                                                 const int32_t *count, double &sum)
{
#pragma unroll
    for (int ox = -1; ox <= 1; ++ox) {
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy) {
#pragma unroll
            for (int oz = 1; oz >= -1; --oz) {
                const int h = ((tx + 1 - ox) * kHY + (ty + 1 - oy)) * kHZ + (tz + 1 - oz);
                const double4 *p = xs + start[h];
                const int32_t cnt = count[h];
                for (int32_t k = 0; k < cnt; ++k) {
                    const double4 r = p[k];
                    double i0;
                    const double dx = tsc_d(r.x, ih, i0), dy = tsc_d(r.y, ih, i0),
                                 dz = tsc_d(r.z, ih, i0);
                    sum += r.w * tsc_w(dx, ox) * tsc_w(dy, oy) * tsc_w_var(dz, oz);
                }
            }
        }
    }
}

// rho at mesh point q: the particles whose nearest point is q - o,
// o in {-1, 0, 1}^3, each with its TSC weight for offset o, summed in a
// fixed order: o_x, then o_y, then o_z = +1, 0, -1, and within a cell the
// sorted order.
// One thread per mesh point of the block's tile.  The particles of the
// tile's neighbourhood go to LDS first (cell by cell, in neighbourhood
// order, with their offsets from the nearest mesh point); a neighbourhood
// with more than kGatherCap particles is read from memory instead, in the
// same order.
__global__ __launch_bounds__(kBlock) void k_gather_rho(int n, double ih, const double4 *xs,
                                                       const int32_t *start,
                                                       const int32_t *end, double *rho)
{
    typedef hipcub::BlockScan<int, kBlock> Scan;
    __shared__ double4 sp[kGatherCap];
    __shared__ uint8_t sz[kGatherCap];  // neighbourhood z index (< kHZ) of each particle
    __shared__ int32_t sfirst[kHalo], scount[kHalo], sstart[kHalo];
    __shared__ typename Scan::TempStorage scan_tmp;
    __shared__ int stotal;
    int x0, y0, z0;
    tile_origin(n, x0, y0, z0);
    const int t = threadIdx.x;
    // counts of the neighbourhood's cells; thread t takes entries 3t .. 3t+2
    constexpr int kPer = (kHalo + kBlock - 1) / kBlock;
    int part = 0;
    for (int u = 0; u < kPer; ++u) {
        const int h = kPer * t + u;
        if (h < kHalo) {
            const int64_t c = halo_point(h, n, x0, y0, z0);
            const int32_t s0 = start[c], c0 = end[c] - s0;
            sstart[h] = s0;
            scount[h] = c0;
            part += c0;
        }
    }
    int excl = 0, total = 0;
    Scan(scan_tmp).ExclusiveSum(part, excl, total);
    for (int u = 0; u < kPer; ++u) {
        const int h = kPer * t + u;
        if (h < kHalo) {
            sfirst[h] = excl;
            excl += scount[h];
        }
    }
    if (t == 0) stotal = total;
    __syncthreads();
    const int ntot = stotal;
    const bool local = ntot <= kGatherCap;
    if (local) {
        // entry j of the LDS copy belongs to the last cell h with
        // sfirst[h] <= j (cells before it that are empty share its first
        // entry; cells after it start beyond j); the threads' loads are
        // independent, so they are all in flight at once
        constexpr int kIter = (kGatherCap + kBlock - 1) / kBlock;
#pragma unroll
        for (int u = 0; u < kIter; ++u) {
            const int j = t + u * kBlock;
            if (j < ntot) {
                int lo = 0, hi = kHalo;  // sfirst[lo] <= j; hi: past the answer
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (sfirst[mid] <= j)
                        lo = mid;
                    else
                        hi = mid;
                }
                const double4 r = xs[sstart[lo] + (j - sfirst[lo])];
                double i0;
                const double dx = tsc_d(r.x, ih, i0), dy = tsc_d(r.y, ih, i0),
                             dz = tsc_d(r.z, ih, i0);
                sp[j] = make_double4(dx, dy, dz, r.w);
                sz[j] = (uint8_t)(lo % kHZ);
            }
        }
    }
    __syncthreads();
    const int tz = t % kTZ, ty = (t / kTZ) % kTY, tx = t / (kTZ * kTY);
    const int qx = x0 + tx, qy = y0 + ty, qz = z0 + tz;
    if (qx >= n || qy >= n || qz >= n) return;
    double sum = 0.0;
    if (local)
        gather_point_lds(tx, ty, tz, sp, sz, sfirst, scount, sum);
    else
        gather_point_mem(tx, ty, tz, ih, xs, sstart, scount, sum);
    rho[((int64_t)qx * n + qy) * n + qz] = sum;
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

// One term of the 27-point interpolation, in the order of the points.
__device__ __forceinline__ void interp_add(const Tsc &w, int a0, int b, int c, const double4 &v,
                                           double *s4)
{
    const double wt = w.w[a0][0] * w.w[b][1] * w.w[c][2];
    s4[0] += wt * v.x;
    s4[1] += wt * v.y;
    s4[2] += wt * v.z;
    s4[3] += wt * v.w;
}

// The particles of the block's tile of cells (nearest mesh point in the
// tile; a row of the tile along z is a contiguous range of the sorted
// order): 27-point TSC interpolation of the interleaved mesh, whose records
// around the tile are in LDS; each result goes to the particle's input
// index.
__global__ __launch_bounds__(kBlock) void k_interp(int n, const double4 *xs, const int32_t *idx,
                                                   const int32_t *start, const int32_t *end,
                                                   double ih, const double4 *m4, double *a,
                                                   double *pot, int accumulate)
{
    constexpr int kRows = kTX * kTY;
    __shared__ double4 sm[kHalo];
    __shared__ int32_t rlo[kRows], rhi[kRows], rpre[kRows + 1];
    int x0, y0, z0;
    tile_origin(n, x0, y0, z0);
    const int t = threadIdx.x;
#pragma unroll
    for (int u = 0; u < (kHalo + kBlock - 1) / kBlock; ++u) {
        const int h = t + u * kBlock;
        if (h < kHalo) sm[h] = m4[halo_point(h, n, x0, y0, z0)];
    }
    if (t < kRows) {
        rlo[t] = 0x7fffffff;
        rhi[t] = 0;
    }
    __syncthreads();
    {
        // row r = (tx, ty): its particles are those of its non-empty cells
        const int tz = t % kTZ, ty = (t / kTZ) % kTY, tx = t / (kTZ * kTY);
        const int cx = x0 + tx, cy = y0 + ty, cz = z0 + tz;
        if (cx < n && cy < n && cz < n) {
            const int64_t c = ((int64_t)cx * n + cy) * n + cz;
            const int32_t s0 = start[c], e0 = end[c];
            if (e0 > s0) {
                atomicMin(&rlo[tx * kTY + ty], s0);
                atomicMax(&rhi[tx * kTY + ty], e0);
            }
        }
    }
    __syncthreads();
    if (t == 0) {
        int acc = 0;
        for (int r = 0; r < kRows; ++r) {
            rpre[r] = acc;
            acc += rhi[r] > rlo[r] ? rhi[r] - rlo[r] : 0;
        }
        rpre[kRows] = acc;
    }
    __syncthreads();
    const int total = rpre[kRows];
    for (int j = t; j < total; j += kBlock) {
        int r = 0;
        while (rpre[r + 1] <= j) ++r;
        const int64_t k = rlo[r] + (j - rpre[r]);
        const double4 rec = xs[k];
        const double xp[3] = {rec.x, rec.y, rec.z};
        const Tsc w = tsc(xp, ih, n);
        // the particle's cell is in the tile (its sort key was computed by
        // the same function): its neighbourhood entries are (w.i - origin) +
        // (0 .. 2) per axis; a cell outside the tile would read the mesh
        const int hx0 = w.i[0] - x0, hy0 = w.i[1] - y0, hz0 = w.i[2] - z0;
        const bool in = hx0 >= 0 && hx0 < kTX && hy0 >= 0 && hy0 < kTY && hz0 >= 0 &&
                        hz0 < kTZ;
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
        if (in) {
#pragma unroll
            for (int a0 = 0; a0 < 3; ++a0)
#pragma unroll
                for (int b = 0; b < 3; ++b)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        interp_add(w, a0, b, c,
                                   sm[((hx0 + a0) * kHY + (hy0 + b)) * kHZ + (hz0 + c)], s4);
        } else {
#pragma unroll
            for (int a0 = 0; a0 < 3; ++a0)
#pragma unroll
                for (int b = 0; b < 3; ++b)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        interp_add(w, a0, b, c,
                                   m4[((int64_t)wrap(w.i[0] + a0 - 1, n) * n +
                                       wrap(w.i[1] + b - 1, n)) * n + wrap(w.i[2] + c - 1, n)],
                                   s4);
        }
        const int64_t p = idx[k];
        if (accumulate) {
            a[3 * p] += s4[0];
            a[3 * p + 1] += s4[1];
            a[3 * p + 2] += s4[2];
            if (pot) pot[p] += s4[3];
        } else {
            a[3 * p] = s4[0];
            a[3 * p + 1] = s4[1];
            a[3 * p + 2] = s4[2];
            if (pot) pot[p] = s4[3];
        }
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
    hipLaunchKernelGGL(k_gather_rho, dim3(ntiles(n)), dim3(kBlock), 0, s, n, ih,
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
    hipLaunchKernelGGL(k_interp, dim3(ntiles(n)), dim3(kBlock), 0, s, n, pm->xs.as<double4>(),
                       pm->idx2.as<int32_t>(), pm->start.as<int32_t>(), pm->end.as<int32_t>(), ih,
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
