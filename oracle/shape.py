"""Relaxed shape derivative and Hilbertian extension-regularisation (oracle,
test infrastructure only).

Sec. 2.2.5 relaxes the compliance shape derivative (Eq. 14) over the whole
domain D: with a perturbation -w n, J' is the integral over D of
sigma(u):eps(u) w H'_eta(phi) |grad phi| (Eq. 15); the volume constraint's
derivative replaces the strain energy density by -1/V_D (Eq. 16); the
augmented Lagrangian combines them with g_L = sigma:eps + (lambda - Lambda C)/V_D
(Eqs. 17-18).  Sec. 2.2.6 extends the result to a velocity vbar by the weighted
H^1 Riesz problem: int ell^2 grad vbar . grad w + vbar w = L'(-w n) for all w
(Eq. 19), discretised as A_H vbar = g (Eq. 20), with vbar = 0 where the loads
act (Gamma_N).

Readings where the paper is silent:
  * phi, w and vbar are trilinear (Q1) on the voxel hexes, like the
    displacements; each element integral is a 2x2x2 Gauss sum (exact for the
    Q1 products, a quadrature of the H'_eta factor);
  * sigma:eps = eps^T D(E0, nu) eps at the Gauss point, with the solid's
    modulus E0: the strain energy density of the solid (Eq. 14); the ersatz
    weight of Eq. 7 enters the state solve only;
  * H'_eta(t) = (1 + cos(pi t / eta)) / (2 eta) for |t| <= eta, else 0, the
    derivative of Eq. 8;
  * the nodal vector g_a = sum_e sum_q w_q h^3 N_a(q) (c_s s(q) + c_0)
    H'_eta(phi(q)) |grad phi(q)|, with (c_s, c_0) = (1, 0) for J',
    (0, -1/V_D) for C', and (1, (lambda - Lambda C)/V_D) for L';
  * A_H = ell^2 K + M with the Q1 Laplacian K and mass M (2x2x2 Gauss, exact
    on a cube);
  * Gamma_N is the set of nodes where the load vector has a non-zero
    component; there vbar = 0 (identity rows); elsewhere the boundary
    condition is the natural one.

  heaviside, heaviside_prime     Eq. 8 and its derivative
  scalar_element_matrices        Q1 Laplacian and mass on one voxel
  energy_density_gauss           sigma:eps at the Gauss points of every element
  shape_rhs                      the nodal vector of Eqs. 15-17
  hilbert_matrix, hilbert_extend A_H (Eq. 20) and its solve with vbar = 0 on Gamma_N
  gamma_n_nodes                  the Gamma_N node mask of a load vector
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import element, grid


def heaviside(t, eta):
    t = np.asarray(t, dtype=np.float64)
    mid = 0.5 + t / (2.0 * eta) + np.sin(np.pi * t / eta) / (2.0 * np.pi)
    return np.where(t < -eta, 0.0, np.where(t > eta, 1.0, mid))


def heaviside_prime(t, eta):
    t = np.asarray(t, dtype=np.float64)
    return np.where(np.abs(t) <= eta, (1.0 + np.cos(np.pi * t / eta)) / (2.0 * eta), 0.0)


def _gauss():
    pts, wts = np.polynomial.legendre.leggauss(2)
    pts = 0.5 * (pts + 1.0)
    wts = 0.5 * wts
    out = []
    for c, wc in zip(pts, wts):          # z slowest, x fastest
        for b, wb in zip(pts, wts):
            for a, wa in zip(pts, wts):
                out.append(((a, b, c), wa * wb * wc))
    return out


def shape_values(xi, eta, zeta):
    """(8,) trilinear shape functions at a reference point; a = ax + 2 ay + 4 az."""
    r = (xi, eta, zeta)
    v = np.ones(8)
    for a in range(8):
        for d in range(3):
            v[a] *= r[d] if (a >> d) & 1 else 1.0 - r[d]
    return v


def scalar_element_matrices(h):
    """(K, M): 8x8 Q1 Laplacian and mass on the cube [0, h]^3 by 2x2x2 Gauss."""
    K = np.zeros((8, 8))
    M = np.zeros((8, 8))
    for (a, b, c), w in _gauss():
        G = element.shape_gradients(a, b, c, h)
        N = shape_values(a, b, c)
        K += w * h ** 3 * (G @ G.T)
        M += w * h ** 3 * np.outer(N, N)
    return K, M


def energy_density_gauss(u, nelx, nely, nelz, h, E0, nu):
    """(nel, 8) sigma:eps = eps^T D eps at the 8 Gauss points of every element."""
    D = element.constitutive(E0, nu)
    ue = np.asarray(u, dtype=np.float64)[grid.element_dofs(nelx, nely, nelz)]
    out = []
    for (a, b, c), _ in _gauss():
        B = element.strain_matrix(element.shape_gradients(a, b, c, h))
        eps = ue @ B.T
        out.append(np.einsum("ei,ij,ej->e", eps, D, eps))
    return np.stack(out, axis=1)


def shape_rhs(u, phi, nelx, nely, nelz, *, h=1.0, E0=1.0, nu=0.3, eta=2.0, c_s=1.0, c_0=0.0):
    """(nn,) g_a = sum_e sum_q w_q h^3 N_a(q) (c_s s(q) + c_0) H'(phi(q)) |grad phi(q)|."""
    en = grid.element_nodes(nelx, nely, nelz)
    pe = np.asarray(phi, dtype=np.float64)[en]
    s = energy_density_gauss(u, nelx, nely, nelz, h, E0, nu) if c_s != 0.0 else None
    g = np.zeros((nelx + 1) * (nely + 1) * (nelz + 1))
    for q, ((a, b, c), w) in enumerate(_gauss()):
        N = shape_values(a, b, c)
        G = element.shape_gradients(a, b, c, h)
        pq = pe @ N
        gq = pe @ G
        dens = c_0 if s is None else c_s * s[:, q] + c_0
        f = w * h ** 3 * dens * heaviside_prime(pq, eta) * np.sqrt(np.sum(gq * gq, axis=1))
        np.add.at(g, en, f[:, None] * N[None, :])
    return g


def hilbert_matrix(nelx, nely, nelz, h, ell):
    """CSR nn x nn A_H = ell^2 K + M assembled from the element matrices."""
    K, M = scalar_element_matrices(h)
    Ae = ell * ell * K + M
    en = grid.element_nodes(nelx, nely, nelz)
    rows = np.repeat(en, 8, axis=1).ravel()
    cols = np.tile(en, (1, 8)).ravel()
    vals = np.tile(Ae.ravel(), en.shape[0])
    nn = (nelx + 1) * (nely + 1) * (nelz + 1)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nn, nn))


def gamma_n_nodes(f):
    """(nn,) bool: nodes with a non-zero load component (f interleaved 3n + c)."""
    return np.any(np.asarray(f, dtype=np.float64).reshape(-1, 3) != 0.0, axis=1)


def hilbert_extend(g, nelx, nely, nelz, *, h=1.0, ell=1.0, dirichlet=None):
    """vbar with A_H vbar = g on the free nodes and vbar = 0 on the Dirichlet
    nodes (sparse direct solve)."""
    A = hilbert_matrix(nelx, nely, nelz, h, ell)
    g = np.asarray(g, dtype=np.float64)
    free = np.ones(g.size, bool) if dirichlet is None else ~np.asarray(dirichlet, bool)
    v = np.zeros(g.size)
    idx = np.flatnonzero(free)
    v[idx] = spla.spsolve(A[idx][:, idx].tocsc(), g[idx])
    return v
