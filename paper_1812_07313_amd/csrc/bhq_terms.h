// bhq_terms.h -- the interaction terms of the Plummer-softened force
// kernels (device code): a particle (or monopole cell) term and a cell term
// with the traceless quadrupole (Kodama & Ishiyama, Sec. 3, eqs. 1, 4-7).
// Shared by the force kernels and the probe that measures their issue rate.
#pragma once

#include <hip/hip_runtime.h>

namespace bhq {

template <typename R>
struct alignas(4 * sizeof(R)) V4 {
    R x, y, z, w;
};

__device__ __forceinline__ float rsq(float v) { return __builtin_amdgcn_rsqf(v); }

// FP64 1/sqrt(v) for finite v > 0 (every argument here: softened r^2 >= eps^2
// > 0, or a split pair's r^2 > 0): the hardware estimate y, then one step of
// the series (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + ... with e = 1 - v y^2, which
// takes the estimate's relative error d to O(d^3).  No special-value handling
// (zero, infinity, denormals), which the library function spends three more
// operations on.
__device__ __forceinline__ double rsq(double v)
{
    const double y = __builtin_amdgcn_rsq(v);
    const double e = fma(-v * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

// Plummer-softened particle (also the monopole-only cell).
template <typename R>
__device__ __forceinline__ void pp_plummer(const V4<R> &j, R xi, R yi, R zi,
                                           R e2, R &ax, R &ay, R &az, R &pt)
{
    const R dx = j.x - xi, dy = j.y - yi, dz = j.z - zi;
    const R r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
    const R rinv = rsq(r2);
    const R mr = j.w * rinv;
    const R mr3 = mr * (rinv * rinv);
    pt += mr;
    ax = fma(mr3, dx, ax);
    ay = fma(mr3, dy, ay);
    az = fma(mr3, dz, az);
}

// Monopole + traceless quadrupole cell (Sec. 3, eqs. 1, 4-7).
// a: (x, y, z, M), b: (q00, q01, q02, q11), c: (q12, q22, T, 0).
// SOFT: the complete second-order expansion of the softened potential,
// which adds T eps^2 / (2 rhat^5) to -phi's quadrupole part with the sign
// of -d.Q.d: d.Q.d becomes d.Q.d - T eps^2 in both terms (one more FMA).
template <typename R, bool SOFT>
__device__ __forceinline__ void pc_quad(const V4<R> &a, const V4<R> &b,
                                        const V4<R> &c, R xi, R yi, R zi, R e2,
                                        R &ax, R &ay, R &az, R &pt)
{
    const R dx = a.x - xi, dy = a.y - yi, dz = a.z - zi;
    const R r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
    const R rinv = rsq(r2);
    const R rinv2 = rinv * rinv;
    const R phim = a.w * rinv;
    const R qx = fma(b.z, dz, fma(b.y, dy, b.x * dx));
    const R qy = fma(c.x, dz, fma(b.w, dy, b.y * dx));
    const R qz = fma(c.y, dz, fma(c.x, dy, b.z * dx));
    R dqd = fma(dz, qz, fma(dy, qy, dx * qx));
    if (SOFT) dqd = fma(-e2, c.z, dqd);
    const R rinv5 = (rinv2 * rinv2) * rinv;
    const R pq = dqd * rinv5;  // 2 phi_quad
    pt += phim;
    pt = fma(R(0.5), pq, pt);
    const R cf = fma(R(2.5), pq, phim) * rinv2;
    ax = fma(cf, dx, ax);
    ay = fma(cf, dy, ay);
    az = fma(cf, dz, az);
    ax = fma(-rinv5, qx, ax);
    ay = fma(-rinv5, qy, ay);
    az = fma(-rinv5, qz, az);
}

}  // namespace bhq
