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
