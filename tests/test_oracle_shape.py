"""Pins for the oracle's relaxed shape derivative (Sec. 2.2.5, Eqs. 15-18) and
Hilbertian extension (Sec. 2.2.6, Eqs. 19-20).

  * the shape functions are isoparametric on the local node order and
    differentiate to the stiffness gradients;
  * the element Laplacian and mass equal their tensor-product closed forms
    (1D stiffness [[1,-1],[-1,1]]/h and mass [[2,1],[1,2]] h/6);
  * H'_eta is the derivative of H_eta (Eq. 8) and integrates to 1;
  * for an affine displacement the Gauss-point energy density is
    eps:C:eps = lambda tr(eps)^2 + 2 mu eps:eps, and over a plane phi = x - x0
    (|grad phi| = 1, band inside the box) the nodal vector sums to s A and to
    c_0 A: the relaxation recovers the boundary integral; the nodal profile
    reduces to a 1D sum, and |grad phi| = 2 leaves the integral unchanged;
  * a manufactured Riesz problem, vbar = cos(pi x/Lx) cos(pi y/Ly) (natural
    conditions on every face), is solved to second order in h;
  * vbar vanishes on Gamma_N, the loaded nodes."""
import numpy as np
import pytest

from oracle import shape as S, element, grid, fem


def test_element_matrices_closed_form():
    for h in (1.0, 0.7):
        K, M = S.scalar_element_matrices(h)
        k1 = np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
        m1 = np.array([[2.0, 1.0], [1.0, 2.0]]) * h / 6.0
        kron3 = lambda a, b, c: np.kron(a, np.kron(b, c))   # z, y, x: x fastest
        assert np.max(np.abs(K - (kron3(m1, m1, k1) + kron3(m1, k1, m1) + kron3(k1, m1, m1)))) < 1e-15
        assert np.max(np.abs(M - kron3(m1, m1, m1))) < 1e-16
        assert abs(M.sum() - h ** 3) < 1e-15 and np.max(np.abs(K.sum(axis=1))) < 1e-15


def test_shape_values_isoparametric():
    # local node a sits at (a & 1, (a >> 1) & 1, (a >> 2) & 1): the shape
    # functions reproduce the reference point and differentiate to the
    # gradients of the element stiffness
    corners = np.array([[a & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], float)
    rng = np.random.default_rng(2)
    for r in rng.uniform(0.0, 1.0, (5, 3)):
        N = S.shape_values(*r)
        assert abs(N.sum() - 1.0) < 1e-15
        assert np.max(np.abs(N @ corners - r)) < 1e-15
        d = 1e-6
        fd = np.stack([(S.shape_values(*(r + d * e)) - S.shape_values(*(r - d * e))) / (2 * d)
                       for e in np.eye(3)], axis=1)
        assert np.max(np.abs(fd - element.shape_gradients(*r, 1.0))) < 1e-9


def test_heaviside_derivative():
    eta = 1.3
    t = np.linspace(-2.0, 2.0, 4001)
    d = 1e-6
    fd = (S.heaviside(t + d, eta) - S.heaviside(t - d, eta)) / (2 * d)
    inside = np.abs(np.abs(t) - eta) > 1e-3
    assert np.max(np.abs(fd - S.heaviside_prime(t, eta))[inside]) < 1e-7
    tt = np.linspace(-3.0, 3.0, 600001)
    assert abs(np.trapezoid(S.heaviside_prime(tt, eta), tt) - 1.0) < 1e-9
    assert abs(S.heaviside(-eta, eta)) < 1e-15 and abs(S.heaviside(eta, eta) - 1.0) < 1e-15
    assert S.heaviside_prime(0.0, eta) == 1.0 / eta


def _affine():
    eps0 = np.array([[1e-2, 2e-3, 0.0], [2e-3, -3e-3, 1e-3], [0.0, 1e-3, 4e-3]])
    lam, mu = element.lame(1.0, 0.3)
    s0 = lam * np.trace(eps0) ** 2 + 2.0 * mu * np.sum(eps0 * eps0)
    return eps0, s0


@pytest.mark.parametrize("eta,x0", [(1.0, 7.3), (2.0, 10.0), (3.0, 8.6)])
def test_plane_recovers_boundary_integral(eta, x0):
    nelx, nely, nelz = 20, 6, 5
    X = grid.node_coords(nelx, nely, nelz, 1.0)
    eps0, s0 = _affine()
    u = (X @ eps0.T).ravel()
    s = S.energy_density_gauss(u, nelx, nely, nelz, 1.0, 1.0, 0.3)
    assert np.max(np.abs(s - s0)) < 1e-14 * s0
    phi = X[:, 0] - x0
    area = nely * nelz
    g = S.shape_rhs(u, phi, nelx, nely, nelz, eta=eta)
    assert abs(g.sum() / (s0 * area) - 1.0) < 1e-13 and np.all(g >= 0.0)
    g0 = S.shape_rhs(u, phi, nelx, nely, nelz, eta=eta, c_s=0.0, c_0=-0.25)
    assert abs(g0.sum() / (-0.25 * area) - 1.0) < 1e-13
    # linear in (c_s, c_0), quadratic in u, zero outside the band's elements
    g2 = S.shape_rhs(2.0 * u, phi, nelx, nely, nelz, eta=eta, c_s=1.0, c_0=-0.25)
    assert np.max(np.abs(g2 - (4.0 * g + g0))) < 1e-15
    far = np.abs(phi) > eta + 1.0
    assert np.all(g[far] == 0.0)


def test_plane_profile_and_gradient_factor():
    # phi = x - x0 depends on x alone and s is uniform, so on nodes away from
    # the y and z faces g reduces to a 1D sum: s h^2 times, over the two
    # elements beside node i and their two Gauss abscissae, w h N1(xi) H'(x - x0)
    nelx, nely, nelz = 16, 5, 4
    h, eta, x0 = 1.0, 2.0, 6.4
    X = grid.node_coords(nelx, nely, nelz, h)
    eps0, s0 = _affine()
    u = (X @ eps0.T).ravel()
    g = S.shape_rhs(u, X[:, 0] - x0, nelx, nely, nelz, eta=eta).reshape(nelz + 1, nely + 1, nelx + 1)
    xg = 0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)
    g1 = np.zeros(nelx + 1)
    for e in range(nelx):
        for xi in xg:
            hp = S.heaviside_prime((e + xi) * h - x0, eta)
            g1[e] += 0.5 * h * (1.0 - xi) * hp
            g1[e + 1] += 0.5 * h * xi * hp
    inner = g[1:-1, 1:-1, :]
    assert np.max(np.abs(inner - s0 * h * h * g1[None, None, :])) < 1e-15
    # |grad phi| = 2: the change of variables leaves the integral unchanged
    g2 = S.shape_rhs(u, 2.0 * (X[:, 0] - x0), nelx, nely, nelz, eta=eta)
    assert abs(g2.sum() / (s0 * nely * nelz) - 1.0) < 1e-3


def test_shape_rhs_scales_with_h():
    # on h = 0.5 the same plane (in element units) carries a quarter of the area
    nelx, nely, nelz = 12, 4, 4
    for h in (1.0, 0.5):
        X = grid.node_coords(nelx, nely, nelz, h)
        eps0, s0 = _affine()
        u = (X @ eps0.T).ravel()
        phi = X[:, 0] - 5.5 * h
        g = S.shape_rhs(u, phi, nelx, nely, nelz, h=h, eta=2.0 * h)
        assert abs(g.sum() / (s0 * nely * nelz * h * h) - 1.0) < 1e-13


def _manufactured(n, ell):
    nelx, nely, nelz = 2 * n, n, 2
    h = 1.0 / n
    Lx, Ly = nelx * h, nely * h
    X = grid.node_coords(nelx, nely, nelz, h)
    c = 1.0 + ell * ell * np.pi ** 2 * (1.0 / Lx ** 2 + 1.0 / Ly ** 2)
    # g_a = int f N_a by 4x4x4 Gauss per element, f = c cos(pi x/Lx) cos(pi y/Ly)
    pts, wts = np.polynomial.legendre.leggauss(4)
    pts, wts = 0.5 * (pts + 1.0), 0.5 * wts
    en = grid.element_nodes(nelx, nely, nelz)
    base = X[en[:, 0]]
    g = np.zeros(X.shape[0])
    for a, wa in zip(pts, wts):
        for b, wb in zip(pts, wts):
            for cz, wc in zip(pts, wts):
                x = base[:, 0] + a * h
                y = base[:, 1] + b * h
                f = c * np.cos(np.pi * x / Lx) * np.cos(np.pi * y / Ly)
                N = S.shape_values(a, b, cz)
                np.add.at(g, en, (wa * wb * wc * h ** 3 * f)[:, None] * N[None, :])
    v = S.hilbert_extend(g, nelx, nely, nelz, h=h, ell=ell)
    exact = np.cos(np.pi * X[:, 0] / Lx) * np.cos(np.pi * X[:, 1] / Ly)
    return np.max(np.abs(v - exact))


def test_manufactured_riesz_second_order():
    for ell in (0.1, 0.4):
        e1, e2 = _manufactured(6, ell), _manufactured(12, ell)
        assert e2 < 0.02 and 3.0 < e1 / e2 < 5.0


def test_dirichlet_on_loaded_nodes():
    nelx, nely, nelz = 8, 3, 3
    fixed, f = fem.problem_arrays(nelx, nely, nelz, grid.BC_CANTILEVER)
    gn = S.gamma_n_nodes(f)
    X = grid.node_coords(nelx, nely, nelz, 1.0)
    assert np.array_equal(np.flatnonzero(gn), np.flatnonzero((X[:, 0] == nelx) & (X[:, 2] == 0)))
    g = np.random.default_rng(0).uniform(0.5, 1.0, X.shape[0])
    v = S.hilbert_extend(g, nelx, nely, nelz, ell=1.0, dirichlet=gn)
    assert np.all(v[gn] == 0.0) and np.all(v[~gn] > 0.0)
    A = S.hilbert_matrix(nelx, nely, nelz, 1.0, 1.0).toarray()
    assert np.max(np.abs(A - A.T)) < 1e-15 and np.linalg.eigvalsh(A).min() > 0.0
