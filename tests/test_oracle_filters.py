"""Pins for the oracle's density and sensitivity filters (Sec. 2.1.3, Eq. 4).

The offset-stencil form is checked against an all-pairs centroid-distance loop,
constant preservation, the adjoint identity and closed-form interior weight
sums."""
import math

import numpy as np
import pytest

from oracle import filters


@pytest.mark.parametrize("r", [1.5, 2.0, 2.5])
def test_stencil_matches_all_pairs(r):
    nelx, nely, nelz = 6, 4, 3
    rng = np.random.default_rng(1)
    x = rng.uniform(0.0, 1.0, nelx * nely * nelz)
    dc = -rng.uniform(0.0, 2.0, x.size)
    a = filters.density_filter(x, nelx, nely, nelz, r)
    b = filters.density_filter_bruteforce(x, nelx, nely, nelz, r)
    assert np.max(np.abs(a - b)) < 1e-14
    a = filters.sensitivity_filter(x, dc, nelx, nely, nelz, r)
    b = filters.sensitivity_filter_bruteforce(x, dc, nelx, nely, nelz, r)
    assert np.max(np.abs(a - b)) < 1e-13 * np.abs(b).max()


def test_stencil_sizes_and_interior_sums():
    assert len(filters.stencil(1.5)) == 19
    assert len(filters.stencil(2.0)) == 27
    s15 = sum(w for *_, w in filters.stencil(1.5))
    s20 = sum(w for *_, w in filters.stencil(2.0))
    assert abs(s15 - (1.5 + 6 * 0.5 + 12 * (1.5 - math.sqrt(2)))) < 1e-15
    assert abs(s15 - 5.529437251522859) < 1e-14
    assert abs(s20 - (2 + 6 * 1 + 12 * (2 - math.sqrt(2)) + 8 * (2 - math.sqrt(3)))) < 1e-14
    assert abs(s20 - 17.173030790971836) < 1e-13
    cnt = filters.neighbour_counts(5, 5, 5, 1.5).reshape(5, 5, 5)
    assert cnt[2, 2, 2] == 19 and cnt[0, 0, 0] == 7    # corner: self + 3 faces + 3 edges


@pytest.mark.parametrize("r", [1.5, 2.0])
def test_constant_preservation_and_adjoint(r):
    nelx, nely, nelz = 7, 5, 4
    rng = np.random.default_rng(2)
    c = np.full(nelx * nely * nelz, 0.37)
    assert np.allclose(filters.density_filter(c, nelx, nely, nelz, r), 0.37, rtol=0, atol=1e-15)
    x = rng.standard_normal(c.size)
    y = rng.standard_normal(c.size)
    lhs = filters.density_filter(x, nelx, nely, nelz, r) @ y
    rhs = x @ filters.density_filter_adjoint(y, nelx, nely, nelz, r)
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)


def test_sensitivity_filter_uniform_density_is_weighted_mean():
    """With rho uniform (>= guard), Eq. 4 reduces to a plain H-weighted mean."""
    nelx, nely, nelz = 5, 4, 3
    rng = np.random.default_rng(3)
    dc = rng.standard_normal(nelx * nely * nelz)
    x = np.full(dc.size, 0.6)
    a = filters.sensitivity_filter(x, dc, nelx, nely, nelz, 2.0)
    b = filters.density_filter(dc, nelx, nely, nelz, 2.0)
    assert np.max(np.abs(a - b)) < 1e-14
