"""Seeded synthetic particle sets (inputs only; no force arithmetic here).

These stand in for the paper's workloads (homogeneous sphere, Plummer model;
Sec. 4 and Sec. 5) and for the five benchmark configurations.  Each
generator takes an explicit seed and returns FP64 positions ``x[n, 3]`` and
masses ``m[n]`` with total mass 1 and G = 1.

Sampling recipes (the paper gives none):
  * Plummer: radius by inverse CDF r = a (X^(-2/3) - 1)^(-1/2) with
    X ~ U(0, 0.999) (so r_max ~ 38.7 a), isotropic direction.
  * uniform cube: U[0, 1)^3 drawn as float32 (values exactly representable
    in FP32), stored as FP64.
  * clustered: 512 Plummer spheres holding 90% of the particles, masses
    from dN/dM ~ M^-1.9 on [1, 1000], scale radius 0.02 (M / M_max)^(1/3),
    centres uniform in [0, 1)^3, particle counts proportional to mass
    (largest remainder, at least one each), plus a 10% uniform background.
  * batched: independent Plummer systems with N = round(2^U),
    U ~ U[10, 16]; each system has total mass 1 and its own softening
    eps = 1 / (4 N^(1/3)).
  * perturbed lattice: the 256^3 grid q = (i + 1/2) / 256 (for n = 2^24),
    x = (q + N(0, sigma^2)) mod 1 in the periodic unit box.
"""
import numpy as np

SEED_BASE = 1812073130


def rng(config_index, sub=0):
    """Generator for configuration k (0-based); sub-streams for batches."""
    return np.random.Generator(np.random.PCG64(SEED_BASE + config_index + sub))


def _isotropic(g, n):
    mu = g.uniform(-1.0, 1.0, n)
    ph = g.uniform(0.0, 2.0 * np.pi, n)
    s = np.sqrt(1.0 - mu * mu)
    return np.stack([s * np.cos(ph), s * np.sin(ph), mu], axis=1)


def plummer(n, g, a=1.0, mass=1.0, xmax=0.999):
    X = g.uniform(0.0, xmax, n)
    X = np.maximum(X, 1e-300)
    r = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    x = r[:, None] * _isotropic(g, n)
    m = np.full(n, mass / n)
    return x, m


def uniform_cube(n, g):
    x = g.random((n, 3), dtype=np.float32).astype(np.float64)
    m = np.full(n, 1.0 / n)
    return x, m


def uniform_sphere(n, g, radius=1.0):
    r = radius * g.random(n) ** (1.0 / 3.0)
    x = r[:, None] * _isotropic(g, n)
    return x, np.full(n, 1.0 / n)


def cold_sphere(n, g, virial=0.1):
    """Homogeneous sphere of radius 1 and mass 1 (G = 1) with isotropic
    Gaussian velocities (zero mean) scaled to the virial ratio
    2K/|W| = virial, |W| = 3/5 being the homogeneous sphere's potential
    energy: the initial state of the cold-collapse runs."""
    x, m = uniform_sphere(n, g)
    v = g.normal(size=(n, 3))
    v -= v.mean(axis=0)
    k = 0.5 * np.sum(m * (v * v).sum(axis=1))
    v *= np.sqrt(virial * 0.6 / (2.0 * k))
    return x, v, m


def clustered(n, g, nclusters=512, slope=1.9, mratio=1000.0, a_max=0.02,
              background=0.1):
    n_bg = int(round(background * n))
    n_cl = n - n_bg
    # dN/dM ~ M^-slope on [1, mratio] by inverse CDF
    u = g.random(nclusters)
    p = 1.0 - slope
    M = (1.0 + u * (mratio ** p - 1.0)) ** (1.0 / p)
    # counts proportional to mass, largest remainder, at least 1 each
    share = M / M.sum() * (n_cl - nclusters)
    cnt = np.floor(share).astype(np.int64)
    rem = (n_cl - nclusters) - cnt.sum()
    order = np.argsort(-(share - cnt), kind="stable")
    cnt[order[:rem]] += 1
    cnt += 1
    centres = g.random((nclusters, 3))
    radii = a_max * (M / M.max()) ** (1.0 / 3.0)
    parts = []
    for k in range(nclusters):
        xk, _ = plummer(int(cnt[k]), g, a=radii[k])
        parts.append(xk + centres[k])
    parts.append(g.random((n_bg, 3)))
    x = np.concatenate(parts, axis=0)
    return x, np.full(n, 1.0 / n)


def batched_sizes(nsys, g, lo=10.0, hi=16.0):
    return np.rint(2.0 ** g.uniform(lo, hi, nsys)).astype(np.int64)


def batched_plummer(nsys, config_index=3, lo=10.0, hi=16.0):
    """List of (x, m, eps) per system; system s uses sub-stream 1000 + s."""
    sizes = batched_sizes(nsys, rng(config_index), lo, hi)
    out = []
    for s, ns in enumerate(sizes):
        x, m = plummer(int(ns), rng(config_index, 1000 + s))
        out.append((x, m, 1.0 / (4.0 * float(ns) ** (1.0 / 3.0))))
    return out


def perturbed_lattice(nside, g, sigma=0.02):
    i = (np.arange(nside, dtype=np.float64) + 0.5) / nside
    q = np.stack(np.meshgrid(i, i, i, indexing="ij"), axis=-1).reshape(-1, 3)
    x = np.mod(q + g.normal(0.0, sigma, q.shape), 1.0)
    x[x >= 1.0] = 0.0
    n = x.shape[0]
    return x, np.full(n, 1.0 / n)


# Named workloads -----------------------------------------------------------

def config_plummer_16k(n=16384):
    """Plummer sphere, N = 16384, eps = 1/64, theta = 0.5, ncrit = 64."""
    x, m = plummer(n, rng(0))
    return dict(x=x, m=m, eps=1.0 / 64.0, theta=0.5, ncrit=64)


def config_uniform_cube(n=1 << 20, theta=0.5):
    """Uniform cube [0,1)^3 (float32 draws), eps = 1e-3, ncrit = 256."""
    x, m = uniform_cube(n, rng(1))
    return dict(x=x, m=m, eps=1e-3, theta=theta, ncrit=256)


def config_clustered(n=1 << 22):
    """512 Plummer clusters + 10% background, eps = 2e-4, theta = 0.5."""
    x, m = clustered(n, rng(2))
    return dict(x=x, m=m, eps=2e-4, theta=0.5, ncrit=256)


def config_lattice(nside=256):
    """Perturbed lattice in the periodic unit box for the short-range split
    kernel: r_s = 1.25 / 256, cutoff 4.5 r_s, theta = 0.5."""
    x, m = perturbed_lattice(nside, rng(4))
    rs = 1.25 / 256.0
    return dict(x=x, m=m, rs=rs, rcut=4.5 * rs, theta=0.5, box=1.0)
