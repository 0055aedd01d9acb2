"""Pins for the oracle's density -> SDF transfer (Secs. 3.2-3.4, Eqs. 25-30)
and the ersatz volume fraction.

Independent checks: linear reproduction of the LSQ map (stated in Sec. 3.2),
its reduction to the mean on voxels, a watertight iso-surface, the exact SDF of
a planar interface, closest points against dense sampling and the KKT
conditions of Eq. 28, a sphere sanity bound, and volume fractions against
closed forms and Monte Carlo."""
import numpy as np
import pytest

from oracle import grid, sdf


def test_lsq_reproduces_linear_field_at_interior_nodes():
    nelx, nely, nelz, h = 5, 4, 3, 0.5
    c = grid.element_centroids(nelx, nely, nelz, h)
    a = np.array([0.3, 0.2, -0.1, 0.4])
    x = a[0] + c @ a[1:]
    rho = sdf.nodal_density_lsq(x, nelx, nely, nelz, h)
    X = grid.node_coords(nelx, nely, nelz, h)
    exact = a[0] + X @ a[1:]
    inner = ((X[:, 0] > 0) & (X[:, 0] < nelx * h) & (X[:, 1] > 0) & (X[:, 1] < nely * h)
             & (X[:, 2] > 0) & (X[:, 2] < nelz * h))
    assert np.max(np.abs(rho[inner] - exact[inner])) < 1e-14


def test_lsq_equals_mean_on_voxels():
    nelx, nely, nelz = 5, 4, 3
    x = np.random.default_rng(0).uniform(0, 1, nelx * nely * nelz)
    a = sdf.nodal_density_lsq(x, nelx, nely, nelz)
    b = sdf.nodal_density_mean(x, nelx, nely, nelz)
    assert np.max(np.abs(a - b)) < 1e-14


def test_kuhn_split_fills_cube():
    vols = []
    for t in sdf.KUHN:
        P = np.array([[(a & 1), (a >> 1) & 1, (a >> 2) & 1] for a in t], dtype=float)
        vols.append(sdf._tet_volume(*P))
    assert np.allclose(vols, 1.0 / 6.0) and len(set(sdf.KUHN)) == 6


def _sphere_density(nelx, nely, nelz, h, center, R, width=1.0):
    c = grid.element_centroids(nelx, nely, nelz, h)
    r = np.linalg.norm(c - np.asarray(center)[None, :], axis=1)
    return 1.0 / (1.0 + np.exp((r - R) / (width * h)))


def test_isosurface_is_watertight():
    nelx = nely = nelz = 8
    x = _sphere_density(nelx, nely, nelz, 1.0, (4.1, 3.9, 4.2), 2.6)
    rho = sdf.nodal_density_mean(x, nelx, nely, nelz)
    T, owner, counts = sdf.marching_tets(rho, nelx, nely, nelz)
    assert counts.sum() == len(T) > 0
    keys = {}
    for tri in T:
        v = [tuple(np.round(p, 12)) for p in tri]
        for a, b in ((0, 1), (1, 2), (2, 0)):
            e = tuple(sorted((v[a], v[b])))
            keys[e] = keys.get(e, 0) + 1
    assert set(keys.values()) == {2}


def test_planar_interface_exact_sdf():
    nelx, nely, nelz, h = 10, 4, 4, 1.0
    x0, s = 4.3, 0.1
    c = grid.element_centroids(nelx, nely, nelz, h)
    x = 0.5 + s * (c[:, 0] - x0)
    phi, rho, vf, T, counts = sdf.density_to_sdf(x, nelx, nely, nelz, h)
    X = grid.node_coords(nelx, nely, nelz, h)
    assert np.max(np.abs(phi - (x0 - X[:, 0]))) < 1e-13
    # solid (phi < 0) is x > x0: exact slab fractions
    ic = np.arange(nelx)
    exact = np.clip((ic + 1) * h - x0, 0, h) / h
    assert np.max(np.abs(vf.reshape(nelz, nely, nelx) - exact[None, None, :])) < 1e-13


def test_closest_point_against_sampling_and_kkt():
    rng = np.random.default_rng(5)
    w = np.linspace(0, 1, 161)
    L2, L3 = np.meshgrid(w, w)
    keep = (L2 + L3) <= 1
    L2, L3 = L2[keep], L3[keep]
    for _ in range(60):
        tri = rng.standard_normal((3, 3))
        if rng.uniform() < 0.2:         # near-degenerate sliver
            tri[2] = tri[0] + 1e-9 * rng.standard_normal(3) + 0.5 * (tri[1] - tri[0])
        xp = rng.standard_normal(3) * 1.5
        d2 = sdf.closest_point_dist2(xp, tri)
        pts = tri[0] + L2[:, None] * (tri[1] - tri[0]) + L3[:, None] * (tri[2] - tri[0])
        samp = np.min(((pts - xp) ** 2).sum(1))
        assert d2 <= samp + 1e-12
        spacing = np.max(np.linalg.norm(tri - tri[[1, 2, 0]], axis=1)) / 160
        assert np.sqrt(samp) - np.sqrt(d2) <= 2 * spacing
        assert d2 <= min(((tri - xp) ** 2).sum(1)) + 1e-15
    # interior projection: residual orthogonal to the plane
    tri = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0]])
    assert abs(sdf.closest_point_dist2(np.array([0.2, 0.3, 0.7]), tri) - 0.49) < 1e-15
    # edge and vertex regions
    assert abs(sdf.closest_point_dist2(np.array([0.5, -2.0, 0.0]), tri) - 4.0) < 1e-15
    assert abs(sdf.closest_point_dist2(np.array([-1.0, -1.0, 1.0]), tri) - 3.0) < 1e-15


def test_vectorised_and_loop_distances_agree():
    nelx = nely = nelz = 5
    x = _sphere_density(nelx, nely, nelz, 1.0, (2.4, 2.6, 2.5), 1.7)
    rho = sdf.nodal_density_mean(x, nelx, nely, nelz)
    T, _, _ = sdf.marching_tets(rho, nelx, nely, nelz)
    P = grid.node_coords(nelx, nely, nelz, 1.0)[::7]
    assert np.max(np.abs(sdf.unsigned_distance(P, T) - sdf.unsigned_distance_vec(P, T))) < 1e-14


def test_sphere_sdf_sanity():
    n, h = 12, 1.0
    cen, R = (6.05, 5.95, 6.1), 3.7
    x = _sphere_density(n, n, n, h, cen, R, width=0.25)
    phi, rho, vf, T, counts = sdf.density_to_sdf(x, n, n, n, h)
    X = grid.node_coords(n, n, n, h)
    exact = np.linalg.norm(X - np.array(cen)[None, :], axis=1) - R
    assert np.max(np.abs(phi - exact)) < 0.5 * h
    assert np.all(np.sign(phi[np.abs(exact) > h]) == np.sign(exact[np.abs(exact) > h]))
    # the node mean of a convex indicator shrinks its 0.5 level set by a
    # fraction of h, so only a coarse volume bound is a sanity check here
    assert abs(vf.sum() * h ** 3 - 4 / 3 * np.pi * R ** 3) < 0.15 * 4 / 3 * np.pi * R ** 3


def test_tet_fraction_closed_forms_and_monte_carlo():
    rng = np.random.default_rng(11)
    P = np.array([[0.0, 0, 0], [1, 0, 0], [1, 1, 0], [1, 1, 1]])
    # sample uniformly in the tet
    u = rng.uniform(size=(200000, 3))
    u.sort(axis=1)
    bary = np.stack([1 - u[:, 2], u[:, 2] - u[:, 1], u[:, 1] - u[:, 0], u[:, 0]], axis=1)
    for nneg in (1, 2, 3):
        F = rng.uniform(0.2, 1.0, 4)
        F[:nneg] *= -1
        rng.shuffle(F)
        got = sdf.tet_negative_fraction(P, F)
        mc = np.mean(bary @ F < 0)
        assert abs(got - mc) < 4e-3
        assert abs(got + sdf.tet_negative_fraction(P, -F) - 1.0) < 1e-14
    assert sdf.tet_negative_fraction(P, np.array([-1.0, -2, -3, -4])) == 1.0
    assert sdf.tet_negative_fraction(P, np.array([1.0, 2, 3, 4])) == 0.0
    # one negative vertex: product of edge fractions
    F = np.array([-1.0, 1.0, 3.0, 1.0])
    assert abs(sdf.tet_negative_fraction(P, F) - 0.5 * 0.25 * 0.5) < 1e-15


def test_triangle_counts_per_voxel_are_bounded():
    rng = np.random.default_rng(2)
    nelx, nely, nelz = 6, 5, 4
    rho = rng.uniform(0, 1, (nelx + 1) * (nely + 1) * (nelz + 1))
    T, owner, counts = sdf.marching_tets(rho, nelx, nely, nelz)
    assert counts.max() <= 12 and counts.sum() == len(T)
    assert np.array_equal(np.bincount(owner, minlength=counts.size), counts)


def test_tet_cases_hand_worked():
    """Sec. 3.3 on one Kuhn tet, worked by hand.  Corners P0..P3 of the
    x-y-z tet with values R; a corner is inside when R >= 0.5.  The cut point
    on edge a -> b (a inside) is P_a + t (P_b - P_a), t = (0.5 - R_a)/(R_b - R_a).

    2 in (0, 1), 2 out (2, 3), R = (1, 3/4, 0, 1/4):
      p_ac: t = 1/2 on P0-P2 -> (1/2, 1/2, 0)
      p_ad: t = 2/3 on P0-P3 -> (2/3, 2/3, 2/3)
      p_bd: t = 1/2 on P1-P3 -> (1, 1/2, 1/2)
      p_bc: t = 1/3 on P1-P2 -> (1, 1/3, 0)
    and the quad is split along p_ac - p_bd: (p_ac, p_ad, p_bd), (p_ac, p_bd, p_bc).
    The four points lie on the level plane 1 - x/4 - 3y/4 + z/4 = 1/2 of the
    tet's linear interpolant, as every marching-tetrahedra quad does, so the
    diagonal changes the triangle list but not the surface."""
    P = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [1, 1, 1]], dtype=float)
    tris = sdf.tet_triangles(P, np.array([1.0, 0.75, 0.0, 0.25]), 0.5)
    pac, pad, pbd, pbc = ([0.5, 0.5, 0.0], [2 / 3, 2 / 3, 2 / 3], [1.0, 0.5, 0.5],
                          [1.0, 1 / 3, 0.0])
    expect = [[pac, pad, pbd], [pac, pbd, pbc]]
    assert len(tris) == 2
    for got, want in zip(tris, expect):
        assert np.max(np.abs(np.array(got) - np.array(want))) <= 1e-15
    level = lambda p: 1 - p[0] / 4 - 3 * p[1] / 4 + p[2] / 4
    for p in (pac, pad, pbd, pbc):
        assert abs(level(p) - 0.5) <= 1e-15
    # 1 in (corner 2), R = (0, 0, 1, 1/4): cuts toward 0, 1, 3 at t = 1/2, 1/2, 2/3
    tris = sdf.tet_triangles(P, np.array([0.0, 0.0, 1.0, 0.25]), 0.5)
    want = [[0.5, 0.5, 0.0], [1.0, 0.5, 0.0], [1.0, 1.0, 2 / 3]]
    assert len(tris) == 1 and np.max(np.abs(np.array(tris[0]) - np.array(want))) <= 1e-15
    # 3 in (0, 1, 3), out 2, R = (1, 1, 0, 3/4): cuts toward 2 at t = 1/2, 1/2, 1/3
    tris = sdf.tet_triangles(P, np.array([1.0, 1.0, 0.0, 0.75]), 0.5)
    want = [[0.5, 0.5, 0.0], [1.0, 0.5, 0.0], [1.0, 1.0, 2 / 3]]
    assert len(tris) == 1 and np.max(np.abs(np.array(tris[0]) - np.array(want))) <= 1e-15
    # all in or all out: nothing
    assert sdf.tet_triangles(P, np.array([1.0, 1.0, 0.5, 0.5]), 0.5) == []
    assert sdf.tet_triangles(P, np.array([0.0, 0.1, 0.2, 0.49]), 0.5) == []
