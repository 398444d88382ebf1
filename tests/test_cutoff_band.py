"""The FP32 split kernels decide the cutoff from FP32 r^2, except for terms
with |r2_32 - fl32(rcut^2)| < band_i, which they decide again from FP64
offsets.  The band is u (16 rcut^2 + 8 |X_i| rcut) with u = 2^-24 and X_i
the i-particle's offset from the group centre: twice the first-order bound
on |r2_32 - |D|^2| near the cutoff.  This checks that bound by emulating the
kernel's FP32 steps (FP32 offsets rounded from FP64 ones, their FP32
difference, r^2 = fma(dz, dz, fma(dy, dy, dx dx))) on random separations
near the cutoff, with i-particles up to several cutoffs from the centre,
and that outside the band the FP32 decision is always the FP64 one."""
import numpy as np

U = 2.0 ** -24


def band(xi32, rcut):
    xn = np.sqrt((xi32.astype(np.float64) ** 2).sum(-1))
    return 2.0 ** -21 * rcut * (2.0 * rcut + xn)


def fma32(a, b, c):
    # a*b is exact in FP64 for FP32 operands; one more rounding to FP32
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def r2_fp32(xj64, xi64):
    xj = xj64.astype(np.float32)
    xi = xi64.astype(np.float32)
    d = (xj - xi).astype(np.float32)
    p = (d[..., 0] * d[..., 0]).astype(np.float32)
    q = fma32(d[..., 1], d[..., 1], p)
    return fma32(d[..., 2], d[..., 2], q)


def test_fp32_cutoff_band_bounds_the_rounding():
    g = np.random.default_rng(7)
    rcut = 4.5 * 1.25 / 256
    n = 400000
    for reach in (0.5, 2.0, 8.0):     # |X_i| up to reach * rcut per axis
        xi = g.uniform(-reach * rcut, reach * rcut, (n, 3))
        u = g.normal(size=(n, 3))
        u /= np.linalg.norm(u, axis=1)[:, None]
        xj = xi + rcut * (1.0 + g.uniform(-3e-6, 3e-6, n))[:, None] * u
        d = xj - xi
        r2_64 = d[:, 2] * d[:, 2] + (d[:, 1] * d[:, 1] + d[:, 0] * d[:, 0])
        r2_32 = r2_fp32(xj, xi).astype(np.float64)
        b = band(xi.astype(np.float32), rcut)
        err = np.abs(r2_32 - r2_64)
        # the error stays within half the band (the band doubles the bound)
        assert np.all(err < 0.5 * b), (reach, float((err / b).max()))
        # outside the band the two decisions agree
        rc2_32 = float(np.float32(rcut * rcut))
        out = np.abs(r2_32 - rc2_32) >= b
        assert np.array_equal((r2_32 < rc2_32)[out], (r2_64 < rcut * rcut)[out])
        # and the band is where they can differ: some decisions inside it do
        inside = ~out
        assert inside.sum() > 1000
        assert np.any((r2_32 < rc2_32)[inside] != (r2_64 < rcut * rcut)[inside])
