"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the method itself: it only produces level
sets sampled on grids, initial and boundary data, the manufactured solution of
section 4.1 with its analytic source terms, and the workload definitions.
Both the oracle and the GPU path consume what it produces.

Model data of eq. (dataeq): a = 1e4, d = 0.1, m_s = 64.06, m_c = 100.09,
porosity phi(c) = 0.01 c + 0.1.
"""
import math

import numpy as np

MODEL = dict(a=1.0e4, d=0.1, m_s=64.06, m_c=100.09, alpha=0.01, beta=0.1)


def grid_axes(n, lo=-1.0, hi=1.0):
    return lo + (hi - lo) * np.arange(n) / (n - 1)


def grid_points(n, dim, lo=-1.0, hi=1.0):
    """Node coordinates in lexicographic order (x fastest), each of shape n^dim."""
    ax = grid_axes(n, lo, hi)
    if dim == 2:
        Y, X = np.meshgrid(ax, ax, indexing="ij")
        return X.reshape(-1), Y.reshape(-1)
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    return X.reshape(-1), Y.reshape(-1), Z.reshape(-1)


# ----------------------------------------------------------------------------
# level sets (inside where phi < 0)
# ----------------------------------------------------------------------------

def disk(n, r=0.4, x0=0.0, y0=0.0):
    x, y = grid_points(n, 2)
    return np.sqrt((x - x0) ** 2 + (y - y0) ** 2) - r


# The paper's Tests 3 and 4 (section 4.2): the box is not printed; [-pi/2, pi/2]^2
# is the reading used here, the smallest symmetric box of this family holding
# both domains (circle radius 1.486, square-with-discs extent 1.2567).
PAPER_BOX = (-math.pi / 2, math.pi / 2)


def paper_circle(n, lo=PAPER_BOX[0], hi=PAPER_BOX[1]):
    """eq. (test13): circle of radius 1.486 centred at (sqrt(2)/30, sqrt(3)/40)."""
    x, y = grid_points(n, 2, lo, hi)
    return np.sqrt((x - math.sqrt(2) / 30) ** 2 + (y - math.sqrt(3) / 40) ** 2) - 1.486


def paper_square(n, lo=PAPER_BOX[0], hi=PAPER_BOX[1], L=0.9567, D=0.3):
    """eq. (test24): union of the square max(|x|, |y|) < L and four discs of radius D
    centred on its vertices."""
    x, y = grid_points(n, 2, lo, hi)
    p1 = np.maximum(np.abs(x), np.abs(y)) - L
    p2 = np.sqrt((np.abs(x) - L) ** 2 + (np.abs(y) - L) ** 2) - D
    return np.minimum(p1, p2)


def necklace_mask(n, beads=8, ring=0.55, radius=0.17):
    """A pixel mask standing in for the paper's image geometries (section 4.3, whose
    images are not available): a ring of eight discs on an n x n grid."""
    x, y = grid_points(n, 2)
    m = np.zeros(n * n, dtype=bool)
    for k in range(beads):
        a = 2 * math.pi * k / beads
        m |= (x - ring * math.cos(a)) ** 2 + (y - ring * math.sin(a)) ** 2 < radius ** 2
    return m


def star(n, a=0.5, b=0.15, k=5, p=0.0):
    x, y = grid_points(n, 2)
    r = np.sqrt(x * x + y * y)
    th = np.arctan2(y, x)          # atan2(0, 0) = 0
    return r - (a + b * np.sin(k * th + p))


def torus(n, R=0.5, r=0.2):
    x, y, z = grid_points(n, 3)
    return np.sqrt((np.sqrt(x * x + y * y) - R) ** 2 + z * z) - r


def ellipsoids(n, centres, semi, smooth=0.02):
    """Union of axis-aligned ellipsoids: the minimum of their scaled level sets, taken as
    a smooth (log-sum-exp) minimum of width `smooth` so that the grooves where two
    ellipsoids meet are rounded instead of creased; smooth=0 gives the plain minimum."""
    x, y, z = grid_points(n, 3)
    qs = []
    for c, s in zip(centres, semi):
        q = np.sqrt(((x - c[0]) / s[0]) ** 2 + ((y - c[1]) / s[1]) ** 2 + ((z - c[2]) / s[2]) ** 2) - 1.0
        qs.append(min(s) * q)
    qs = np.array(qs)
    m = qs.min(axis=0)
    if smooth <= 0.0 or len(qs) == 1:
        return m
    return m - smooth * np.log(np.exp(-(qs - m) / smooth).sum(axis=0))


# ----------------------------------------------------------------------------
# manufactured solution of section 4.1 and its source terms
# ----------------------------------------------------------------------------

SQ2, SQ3 = math.sqrt(2.0), math.sqrt(3.0)


def s_exact(x, y, t):
    return 2.0 + np.sin(x) * np.cos(y) * np.sin(t + SQ2)


def s_exact_grad(x, y, t):
    """(ds/dx, ds/dy) of s_exact, for Neumann boundary data ds/dn = grad s . n."""
    st = np.sin(t + SQ2)
    return np.cos(x) * np.cos(y) * st, -np.sin(x) * np.sin(y) * st


def c_exact(x, y, t):
    return 3.0 + np.sin(0.5 * x) * np.cos(3.0 * y) * np.sin(2.0 * t + SQ3)


def mms_sources(x, y, t, a=MODEL["a"], d=MODEL["d"], m_s=MODEL["m_s"], m_c=MODEL["m_c"],
                alpha=MODEL["alpha"], beta=MODEL["beta"]):
    """f1, f2 such that s_exact, c_exact solve the forced model of section 4.1:
    d(phi s)/dt = -(a/m_c) phi s c + d div(phi grad s) + f1,
    dc/dt = -(a/m_s) phi s c + f2."""
    st = np.sin(t + SQ2)
    s = 2.0 + np.sin(x) * np.cos(y) * st
    s_t = np.sin(x) * np.cos(y) * np.cos(t + SQ2)
    s_x = np.cos(x) * np.cos(y) * st
    s_y = -np.sin(x) * np.sin(y) * st
    lap_s = -2.0 * np.sin(x) * np.cos(y) * st
    ct = np.sin(2.0 * t + SQ3)
    c = 3.0 + np.sin(0.5 * x) * np.cos(3.0 * y) * ct
    c_t = 2.0 * np.sin(0.5 * x) * np.cos(3.0 * y) * np.cos(2.0 * t + SQ3)
    c_x = 0.5 * np.cos(0.5 * x) * np.cos(3.0 * y) * ct
    c_y = -3.0 * np.sin(0.5 * x) * np.sin(3.0 * y) * ct
    por = alpha * c + beta
    f1 = alpha * c_t * s + por * s_t + (a / m_c) * por * s * c - d * (alpha * (c_x * s_x + c_y * s_y) + por * lap_s)
    f2 = c_t + (a / m_s) * por * s * c
    return f1, f2


def sphere(n, r=0.6, centre=(0.0, 0.0, 0.0)):
    """Signed distance to a sphere: the 3-D domain of the manufactured-solution tests."""
    x, y, z = grid_points(n, 3)
    return np.sqrt((x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2) - r


def s_exact3(x, y, z, t):
    """The section 4.1 solution for s with a cos z factor: the 3-D manufactured solution."""
    return 2.0 + np.sin(x) * np.cos(y) * np.cos(z) * np.sin(t + SQ2)


def s_exact3_grad(x, y, z, t):
    st = np.sin(t + SQ2)
    return (np.cos(x) * np.cos(y) * np.cos(z) * st, -np.sin(x) * np.sin(y) * np.cos(z) * st,
            -np.sin(x) * np.cos(y) * np.sin(z) * st)


def c_exact3(x, y, z, t):
    return 3.0 + np.sin(0.5 * x) * np.cos(3.0 * y) * np.cos(z) * np.sin(2.0 * t + SQ3)


def mms_sources3(x, y, z, t, a=MODEL["a"], d=MODEL["d"], m_s=MODEL["m_s"], m_c=MODEL["m_c"],
                 alpha=MODEL["alpha"], beta=MODEL["beta"]):
    """f1, f2 of the forced model (as mms_sources) for s_exact3, c_exact3."""
    st = np.sin(t + SQ2)
    u = np.sin(x) * np.cos(y) * np.cos(z)
    s = 2.0 + u * st
    s_t = u * np.cos(t + SQ2)
    s_x, s_y, s_z = s_exact3_grad(x, y, z, t)
    lap_s = -3.0 * u * st
    ct = np.sin(2.0 * t + SQ3)
    v = np.sin(0.5 * x) * np.cos(3.0 * y) * np.cos(z)
    c = 3.0 + v * ct
    c_t = 2.0 * v * np.cos(2.0 * t + SQ3)
    c_x = 0.5 * np.cos(0.5 * x) * np.cos(3.0 * y) * np.cos(z) * ct
    c_y = -3.0 * np.sin(0.5 * x) * np.sin(3.0 * y) * np.cos(z) * ct
    c_z = -np.sin(0.5 * x) * np.cos(3.0 * y) * np.sin(z) * ct
    por = alpha * c + beta
    f1 = (alpha * c_t * s + por * s_t + (a / m_c) * por * s * c
          - d * (alpha * (c_x * s_x + c_y * s_y + c_z * s_z) + por * lap_s))
    f2 = c_t + (a / m_s) * por * s * c
    return f1, f2


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

CONFIGS = {
    "disk65": dict(kind="disk", dim=2, n=65, coarsest=5, dt=1e-3, steps=10, precision=0),
    "star1025": dict(kind="star", dim=2, n=1025, coarsest=9, dt=1e-4, steps=100, precision=0),
    "torus257": dict(kind="torus", dim=3, n=257, coarsest=9, dt=1e-4, steps=20, precision=1),
}


def levelset_for(cfg):
    if cfg["kind"] == "disk":
        return disk(cfg["n"])
    if cfg["kind"] == "star":
        return star(cfg["n"], **cfg.get("shape", {}))
    if cfg["kind"] == "torus":
        return torus(cfg["n"])
    if cfg["kind"] == "ellipsoids":
        return ellipsoids(cfg["n"], cfg["centres"], cfg["semi"])
    raise ValueError(cfg["kind"])


def initial_state(n, dim, s0=0.0, c0=1.0):
    """Constant initial data on the whole grid (ghost values included)."""
    nn = n ** dim
    return np.full(nn, s0), np.full(nn, c0)


def batch_domains(count=64, seed=0):
    """Star domains with per-domain draws in the order a, b, k, p, n."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        a = rng.uniform(0.35, 0.6)
        b = rng.uniform(0.05, 0.2)
        k = int(rng.integers(3, 9))
        p = rng.uniform(0.0, 2.0 * math.pi)
        n = int(rng.choice([129, 257, 513, 1025]))
        out.append(dict(kind="star", dim=2, n=n, coarsest=9, dt=1e-4, steps=50, precision=1,
                        shape=dict(a=a, b=b, k=k, p=p)))
    return out


def serving_requests(count=64, rate=1.0, seed=0):
    """Poisson stream of ellipsoid-union domains; per request the draws are:
    arrival gap, number of ellipsoids, centres, semi-axes, grid size, steps."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        m = int(rng.integers(1, 5))
        centres = [tuple(rng.uniform(-0.5, 0.5, 3)) for _ in range(m)]
        semi = [tuple(rng.uniform(0.15, 0.45, 3)) for _ in range(m)]
        n = int(rng.choice([65, 129, 257]))
        steps = int(rng.integers(10, 201))
        out.append(dict(id=i, arrival=t, kind="ellipsoids", dim=3, n=n, coarsest=9, dt=1e-4,
                        steps=steps, precision=1, centres=centres, semi=semi))
    return out
