"""FP64 reference of the particle-mesh long-range force that completes the
Gaussian-split short-range tree force into a TreePM force (the paper's
TreePM context, Sec. 1: the tree computes the short-range part, the PM
method the long-range part).

TEST INFRASTRUCTURE ONLY: used by the test suite, never by the library.

With the short-range pair potential -erfc(r / 2 r_s) / r, the long-range
part is -erf(r / 2 r_s) / r, whose Fourier transform is
-4 pi exp(-k^2 r_s^2) / k^2.  In a periodic box of side L (mean density
removed, G = 1):
    phi_long(x) = -(4 pi / L^3) sum_{k != 0} exp(-k^2 r_s^2) / k^2
                   sum_p m_p cos(k . (x - x_p))
    a_long(x)   = -grad phi_long.
`direct_k_sum` evaluates this definition mode by mode (no mesh).  `pm`
evaluates it the particle-mesh way, step by step:
  1. triangular-shaped-cloud (TSC) assignment of the masses to an n^3 mesh
     (mesh points at integer multiples of h = L / n, periodic), one of the
     27 stencil offsets at a time (a weighted histogram per offset);
  2. forward FFT of the density;
  3. multiplication by -4 pi exp(-k^2 r_s^2) / k^2 (k = 0 set to zero)
     and division by the squared TSC window prod_a sinc(k_a h / 2)^6
     (assignment and interpolation);
  4. the gradient in Fourier space, -i k phi(k) (Nyquist planes zero);
  5. inverse FFTs and TSC interpolation back to the particles.
numpy's FFT is the library primitive for steps 2 and 5.
"""
import numpy as np


def tsc_weights(x, h, n):
    """Nearest mesh index i0 (mod n) and the three weights for offsets -1,
    0, +1 along each axis: w = ((1/2 - d)^2 / 2, 3/4 - d^2, (1/2 + d)^2 / 2)
    with d = x/h - round(x/h)."""
    u = np.asarray(x, np.float64) / h
    i0 = np.floor(u + 0.5)
    d = u - i0
    w = np.stack([0.5 * (0.5 - d) ** 2, 0.75 - d * d, 0.5 * (0.5 + d) ** 2], axis=0)
    return i0.astype(np.int64) % n, w


def _k_vectors(n, L):
    k = 2.0 * np.pi * np.fft.fftfreq(n, d=L / n)
    kz = 2.0 * np.pi * np.fft.rfftfreq(n, d=L / n)
    return k, k, kz


def pm(x, m, L, n, rs, deconvolve=True):
    """Long-range acceleration a[N, 3] and potential phi[N] by the
    particle-mesh method on an n^3 mesh (n even)."""
    x = np.asarray(x, np.float64).reshape(-1, 3)
    m = np.asarray(m, np.float64)
    h = L / n
    i0, w = tsc_weights(x, h, n)
    rho = np.zeros(n * n * n)
    for a in range(3):
        for b in range(3):
            for c in range(3):
                flat = (((i0[:, 0] + a - 1) % n) * n + (i0[:, 1] + b - 1) % n) * n \
                    + (i0[:, 2] + c - 1) % n
                rho += np.bincount(flat, weights=m * w[a, :, 0] * w[b, :, 1] * w[c, :, 2],
                                   minlength=n * n * n)
    rho = rho.reshape(n, n, n) / h ** 3
    rk = np.fft.rfftn(rho)
    kx, ky, kz = _k_vectors(n, L)
    KX, KY, KZ = np.meshgrid(kx, ky, kz, indexing="ij")
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        green = -4.0 * np.pi * np.exp(-k2 * rs * rs) / k2
    green[0, 0, 0] = 0.0
    if deconvolve:
        win = (np.sinc(KX * h / (2 * np.pi)) * np.sinc(KY * h / (2 * np.pi))
               * np.sinc(KZ * h / (2 * np.pi))) ** 3
        green = green / win ** 2
    phik = green * rk
    nyq = n // 2
    out = []
    for K, axis in ((KX, 0), (KY, 1), (KZ, 2)):
        Kd = K.copy()
        if axis < 2:
            sl = [slice(None)] * 3
            sl[axis] = nyq
            Kd[tuple(sl)] = 0.0
        else:
            Kd[:, :, nyq] = 0.0
        out.append(np.fft.irfftn(-1j * Kd * phik, s=(n, n, n), axes=(0, 1, 2)))
    phim = np.fft.irfftn(phik, s=(n, n, n), axes=(0, 1, 2))
    meshes = out + [phim]
    res = np.zeros((x.shape[0], 4))
    flat_meshes = [q.ravel() for q in meshes]
    for a in range(3):
        for b in range(3):
            for c in range(3):
                flat = (((i0[:, 0] + a - 1) % n) * n + (i0[:, 1] + b - 1) % n) * n \
                    + (i0[:, 2] + c - 1) % n
                wt = w[a, :, 0] * w[b, :, 1] * w[c, :, 2]
                for q in range(4):
                    res[:, q] += wt * flat_meshes[q][flat]
    return res[:, :3], res[:, 3]


def direct_k_sum(x, xp, mp, L, rs, kmax_factor=6.0):
    """The long-range acceleration and potential at points x of point
    masses mp at xp, by the definition's sum over wave vectors (all k with
    |k| r_s <= kmax_factor, where exp(-k^2 r_s^2) < 3e-16 beyond)."""
    x = np.asarray(x, np.float64).reshape(-1, 3)
    xp = np.asarray(xp, np.float64).reshape(-1, 3)
    mp = np.asarray(mp, np.float64)
    nmax = int(np.ceil(kmax_factor / rs * L / (2 * np.pi)))
    r = np.arange(-nmax, nmax + 1)
    NX, NY, NZ = np.meshgrid(r, r, r, indexing="ij")
    K = 2.0 * np.pi / L * np.stack([NX.ravel(), NY.ravel(), NZ.ravel()], axis=1)
    k2 = (K * K).sum(1)
    keep = (k2 > 0) & (k2 * rs * rs <= kmax_factor ** 2)
    K, k2 = K[keep], k2[keep]
    coef = -4.0 * np.pi / L ** 3 * np.exp(-k2 * rs * rs) / k2
    a = np.zeros((x.shape[0], 3))
    phi = np.zeros(x.shape[0])
    for j in range(xp.shape[0]):
        arg = (x - xp[j]) @ K.T
        phi += mp[j] * (np.cos(arg) @ coef)
        a += mp[j] * ((np.sin(arg) * coef) @ K)
    return a, phi
