"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  Holds no arithmetic of the method itself: it only draws densities.

Random-field densities (the paper's benchmark meshes and densities are not
available; these stand in for SIMP designs of the same shape):
  white noise from numpy's default_rng(seed), shape (nelz, nely, nelx) so that
  the C-order flattening is the element order i + nelx (j + nely k); smoothed
  with a Gaussian of standard deviation `ell` elements (reflecting boundary,
  truncated at 4 sigma); standardised to zero mean and unit deviation; mapped
  to [xmin, 1] by xmin + (1 - xmin) * sigmoid(kappa * (g - shift)).
  kappa = 2 gives smooth "random-field" densities, kappa = 8 gives sharper
  "SIMP-like" ones; `solid_fraction` shifts g so that that fraction of the
  elements has x > 0.5 (the paper's target volume fraction is 0.4).
"""
import numpy as np
from scipy import ndimage


def random_field(nelx, nely, nelz, seed, ell=6.0, kappa=2.0, xmin=1e-3, solid_fraction=None):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((nelz, nely, nelx))
    g = ndimage.gaussian_filter(g, sigma=ell, mode="reflect", truncate=4.0)
    g = (g - g.mean()) / g.std()
    shift = 0.0
    if solid_fraction is not None:
        shift = np.quantile(g, 1.0 - solid_fraction)
    x = xmin + (1.0 - xmin) / (1.0 + np.exp(-kappa * (g - shift)))
    return np.ascontiguousarray(x.ravel(), dtype=np.float64)


def uniform(nelx, nely, nelz, value=0.5):
    return np.full(nelx * nely * nelz, value, dtype=np.float64)


def random_vector(n, seed):
    return np.random.default_rng(seed).standard_normal(n)


def _node_coords(nelx, nely, nelz):
    k, j, i = np.meshgrid(np.arange(nelz + 1), np.arange(nely + 1), np.arange(nelx + 1),
                          indexing="ij")
    return i.ravel().astype(float), j.ravel().astype(float), k.ravel().astype(float)


def sphere_union(nelx, nely, nelz, seed, count=3, scale=1.0):
    """Level-set input on the (nelx+1)(nely+1)(nelz+1) nodes (node order
    i + NX (j + NY k), unit spacing): `scale` times the distance to the union
    of `count` balls with seeded centres and radii, negative inside (an exact
    signed distance outside the balls when scale is 1)."""
    i, j, k = _node_coords(nelx, nely, nelz)
    dims = np.array([nelx, nely, nelz], dtype=float)
    rng = np.random.default_rng(seed)
    phi = np.full(i.size, np.inf)
    for _ in range(count):
        c = rng.uniform(0, 1, 3) * dims
        R = rng.uniform(0.15, 0.3) * dims.min() + 0.7
        phi = np.minimum(phi, np.sqrt((i - c[0]) ** 2 + (j - c[1]) ** 2 + (k - c[2]) ** 2) - R)
    return np.ascontiguousarray(scale * phi)


def smooth_speed(nelx, nely, nelz, seed):
    """A smooth nodal normal speed of both signs, |v| <= 1.3."""
    i, j, k = _node_coords(nelx, nely, nelz)
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.05, 0.4, 4)
    return np.ascontiguousarray(0.8 * np.sin(a[0] * i + 0.3) * np.cos(a[1] * j)
                                + 0.5 * np.sin(a[2] * k + a[3] * j))
