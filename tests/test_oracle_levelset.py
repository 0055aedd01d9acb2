"""Pins for the oracle's level-set evolution and reinitialisation (Sec. 2.2.7,
Eqs. 21-22; Sec. 2.2.8, Eqs. 23-24).

  * hand-worked single steps on a 1D profile (phi = x^2 with v = +1 and -1, a
    slope-2 line under reinitialisation), whose values follow from the
    one-sided differences by hand;
  * planes move exactly by v dt per step on nodes whose stencils never reach
    a box face, for either sign of v and any normal;
  * a constant field is fixed; an axis-aligned signed distance is a fixed
    point of reinitialisation; a slope-2 line whose zero is on a node is
    reinitialised to the exact distance;
  * mirror and axis-permutation invariance (a swapped pairing of one-sided
    differences, or an axis mix-up, breaks them);
  * a sphere given by (r^2 - R^2)/(2R) is brought to within 0.8 h of r - R in
    a band of 3 h, with the stop rule and the step cap."""
import numpy as np
import pytest

from oracle import levelset as LS


def coords(nelx, nely, nelz):
    k, j, i = np.meshgrid(np.arange(nelz + 1), np.arange(nely + 1), np.arange(nelx + 1),
                          indexing="ij")
    return i.ravel().astype(float), j.ravel().astype(float), k.ravel().astype(float)


def test_hand_worked_steps():
    # 5 x 2 x 2 nodes, phi = x^2 along x, h = 1, gamma = 1/2 -> dt = 1/2
    i, _, _ = coords(4, 1, 1)
    phi = i ** 2
    p, dt = LS.advect(phi, np.ones(phi.size), 4, 1, 1, 1.0, 0.5, 1)
    assert dt == 0.5
    # v > 0 takes the backward difference where it is positive: 0, 1, 3, 5, 7
    # at the nodes (the first node has none: the face rule gives 0)
    assert np.array_equal(p[:5], [0.0, 0.5, 2.5, 6.5, 12.5])
    p, _ = LS.advect(phi, -np.ones(phi.size), 4, 1, 1, 1.0, 0.5, 1)
    # v < 0 takes the forward difference where it is positive: 1, 3, 5, 7, 0
    assert np.array_equal(p[:5], [0.5, 2.5, 6.5, 12.5, 16.0])
    # slope-2 line [-4, -2, 0, 2, 4]: at x = 3, S = 2 / sqrt(4 + 2^2) and the
    # upwind slope is 2, so phi = 2 - (1/2)(1/sqrt 2)(2 - 1); at the face
    # x = 4 the central slope is (4 - 2)/2 = 1, S = 4/sqrt(17)
    p = LS.reinit_step(2.0 * (i - 2.0), 4, 1, 1, 1.0, 0.5)
    assert p[2] == 0.0
    assert abs(p[3] - (2.0 - 0.5 / np.sqrt(2.0))) < 1e-15
    assert abs(p[4] - (4.0 - 2.0 / np.sqrt(17.0))) < 1e-15
    assert np.allclose(p[:5], -p[4::-1], rtol=0, atol=1e-15)


@pytest.mark.parametrize("normal,v", [((1, 2, -2), 0.7), ((1, 2, -2), -0.7), ((0, 0, 1), 1.3),
                                      ((-3, 0, 4), -0.4)])
def test_planes_move_exactly_inside(normal, v):
    nelx, nely, nelz = 16, 14, 12
    i, j, k = coords(nelx, nely, nelz)
    n = np.asarray(normal, float) / np.linalg.norm(normal)
    phi = n[0] * i + n[1] * j + n[2] * k - 5.1
    steps, gamma = 3, 0.5
    p, dt = LS.advect(phi, np.full(phi.size, v), nelx, nely, nelz, 1.0, gamma, steps)
    assert dt == gamma / abs(v)
    inside = ((i >= steps) & (i <= nelx - steps) & (j >= steps) & (j <= nely - steps)
              & (k >= steps) & (k <= nelz - steps))
    assert np.max(np.abs(p - (phi - steps * v * dt))[inside]) < 1e-12
    # a face node whose upwind neighbour lies outside the box moves less
    assert np.max(np.abs(p - (phi - steps * v * dt))) > 1e-3 or normal == (0, 0, 1)


def test_constant_and_zero_speed():
    phi = np.full(5 * 4 * 3, 2.5)
    p, dt = LS.advect(phi, np.linspace(-1, 1, phi.size), 4, 3, 2, 1.0, 0.5, 4)
    assert np.array_equal(p, phi)
    rng = np.random.default_rng(0)
    phi = rng.standard_normal(5 * 4 * 3)
    p, dt = LS.advect(phi, np.zeros(phi.size), 4, 3, 2, 1.0, 0.5, 4)
    assert dt == 0.0 and np.array_equal(p, phi)


def test_reinit_fixed_point_and_exact_line():
    nelx, nely, nelz = 20, 6, 5
    i, _, _ = coords(nelx, nely, nelz)
    sdf = i - 7.3
    p, steps, change = LS.reinit(sdf, nelx, nely, nelz, 1.0, 0.5, 1e-12, 10)
    assert steps == 1 and np.max(np.abs(p - sdf)) < 1e-14
    p, steps, _ = LS.reinit(2.0 * (i - 7.0), nelx, nely, nelz, 1.0, 0.5, 1e-12, 2000)
    assert np.max(np.abs(p - (i - 7.0))) < 1e-9
    # zero between nodes: the first-order smeared-sign scheme moves it slightly
    p, steps, _ = LS.reinit(2.0 * (i - 7.3), nelx, nely, nelz, 1.0, 0.5, 1e-12, 2000)
    assert np.max(np.abs(p - (i - 7.3))) < 0.05


def _smooth(nelx, nely, nelz, seed):
    i, j, k = coords(nelx, nely, nelz)
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.2, 0.6, 6)
    return (np.sin(a[0] * i + 1.0) * np.cos(a[1] * j) + 0.5 * np.sin(a[2] * k + a[3] * i)
            + 0.3 * np.cos(a[4] * j + a[5] * k))


def test_mirror_and_axis_permutation_invariance():
    nelx, nely, nelz = 9, 7, 6
    phi = _smooth(nelx, nely, nelz, 1)
    v = _smooth(nelx, nely, nelz, 2)
    g = lambda a: a.reshape(nelz + 1, nely + 1, nelx + 1)
    p, _ = LS.advect(phi, v, nelx, nely, nelz, 1.0, 0.5, 3)
    r = LS.reinit_step(phi, nelx, nely, nelz, 1.0, 0.4)
    for ax in (0, 1, 2):
        pm, _ = LS.advect(np.flip(g(phi), ax).ravel(), np.flip(g(v), ax).ravel(),
                          nelx, nely, nelz, 1.0, 0.5, 3)
        assert np.max(np.abs(g(pm) - np.flip(g(p), ax))) < 1e-14
        rm = LS.reinit_step(np.flip(g(phi), ax).ravel(), nelx, nely, nelz, 1.0, 0.4)
        assert np.max(np.abs(g(rm) - np.flip(g(r), ax))) < 1e-14
    # x <-> z: the array becomes (nelx+1, nely+1, nelz+1) in (k, j, i) order
    tp = lambda a: np.ascontiguousarray(g(a).transpose(2, 1, 0)).ravel()
    pt, _ = LS.advect(tp(phi), tp(v), nelz, nely, nelx, 1.0, 0.5, 3)
    assert np.max(np.abs(pt - tp(p))) < 1e-14
    rt = LS.reinit_step(tp(phi), nelz, nely, nelx, 1.0, 0.4)
    assert np.max(np.abs(rt - tp(r))) < 1e-14


def test_sphere_reinit_band_and_stop_rule():
    nelx, nely, nelz = 24, 20, 16
    i, j, k = coords(nelx, nely, nelz)
    R = 6.0
    r = np.sqrt((i - 11.3) ** 2 + (j - 9.7) ** 2 + (k - 8.2) ** 2)
    phi0 = (r ** 2 - R ** 2) / (2 * R)
    p, steps, change = LS.reinit(phi0, nelx, nely, nelz, 1.0, 0.5, 1e-3, 1000)
    assert change < 1e-3 and 20 < steps < 1000
    band = np.abs(r - R) <= 3.0
    assert np.max(np.abs(p - (r - R))[band]) < 0.8
    assert np.all(np.sign(p[np.abs(r - R) > 1.0]) == np.sign((r - R)[np.abs(r - R) > 1.0]))
    with pytest.raises(RuntimeError):
        LS.reinit(phi0, nelx, nely, nelz, 1.0, 0.5, 1e-3, 5)
    with pytest.raises(ValueError):
        LS.reinit(np.where(r < 2, np.nan, phi0), nelx, nely, nelz)
