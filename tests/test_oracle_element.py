"""Pins for the oracle's unit-modulus hex8 stiffness k_e^0 (Sec. 2.1.2, Eq. 3).

Each check is independent of the Gauss-quadrature B^T D B route the oracle
uses: exact rational integration of the weak form, the rigid-body null space,
the constant-strain energy identity, and closed forms for the diagonal.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import element

pytestmark = pytest.mark.filterwarnings("ignore")


def _int1d(a_bit, b_bit, da, db):
    """Exact int_0^1 f_a^(da) f_b^(db) dt with f_0 = 1 - t, f_1 = t."""
    # f and f' as polynomial coefficient lists [c0, c1]
    f = {0: [Fraction(1), Fraction(-1)], 1: [Fraction(0), Fraction(1)]}
    df = {0: [Fraction(-1)], 1: [Fraction(1)]}
    p = df[a_bit] if da else f[a_bit]
    q = df[b_bit] if db else f[b_bit]
    prod = [Fraction(0)] * (len(p) + len(q) - 1)
    for i, x in enumerate(p):
        for j, y in enumerate(q):
            prod[i + j] += x * y
    return sum(c / (n + 1) for n, c in enumerate(prod))


def _grad_integral(a, b, i, k):
    """Exact int_[0,1]^3 d_i N_a d_k N_b."""
    val = Fraction(1)
    for d in range(3):
        ba, bb = (a >> d) & 1, (b >> d) & 1
        val *= _int1d(ba, bb, d == i, d == k)
    return val


def _exact_A_B():
    A = [[Fraction(0)] * 24 for _ in range(24)]
    B = [[Fraction(0)] * 24 for _ in range(24)]
    for a in range(8):
        for b in range(8):
            gg = sum(_grad_integral(a, b, d, d) for d in range(3))
            for i in range(3):
                for k in range(3):
                    A[3 * a + i][3 * b + k] = 72 * _grad_integral(a, b, i, k)
                    B[3 * a + i][3 * b + k] = 72 * ((gg if i == k else 0) + _grad_integral(a, b, k, i))
    return A, B


def test_k0_equals_exact_weak_form():
    """K0 = (lam A + mu B)/72 with A, B from exact integration of
    lam div u div v + 2 mu eps(u):eps(v); A and B are integer matrices."""
    A, B = _exact_A_B()
    assert all(x.denominator == 1 for row in A + B for x in row)
    nu = Fraction(3, 10)
    lam = nu / ((1 + nu) * (1 - 2 * nu))
    mu = 1 / (2 * (1 + nu))
    Kx = np.array([[float((lam * A[r][c] + mu * B[r][c]) / 72) for c in range(24)] for r in range(24)])
    K = element.k0(0.3, 1.0)
    assert np.max(np.abs(K - Kx)) <= 2e-16 * 4
    # nu = 0.3: K0 = M * 5/1872 with an integer M
    M = [[(lam * A[r][c] + mu * B[r][c]) / 72 / Fraction(5, 1872) for c in range(24)] for r in range(24)]
    assert all(m.denominator == 1 for row in M for m in row)
    assert max(abs(int(m)) for row in M for m in row) == 88


def test_k0_gauss_orders_agree_and_scale_with_h():
    K2 = element.k0(0.3, 1.0, order=2)
    K3 = element.k0(0.3, 1.0, order=3)
    assert np.max(np.abs(K2 - K3)) < 1e-15
    for h in (0.05, 0.5, 3.0):
        assert np.allclose(element.k0(0.3, h), h * K2, rtol=0, atol=1e-15 * h)


def _rigid_modes(h=1.0):
    pos = np.array([[(a & 1) * h, ((a >> 1) & 1) * h, ((a >> 2) & 1) * h] for a in range(8)])
    modes = []
    for c in range(3):
        t = np.zeros((8, 3))
        t[:, c] = 1.0
        modes.append(t.ravel())
    for w in np.eye(3):
        modes.append(np.cross(w[None, :], pos).ravel())
    return np.array(modes)


@pytest.mark.parametrize("nu", [0.0, 0.3, 0.45])
def test_k0_symmetric_psd_six_null_modes(nu):
    K = element.k0(nu, 1.0)
    assert np.array_equal(K, K.T)
    ev = np.linalg.eigvalsh(K)
    assert np.sum(np.abs(ev) < 1e-12) == 6
    assert ev[6] > 1e-3
    R = _rigid_modes()
    assert np.max(np.abs(K @ R.T)) < 1e-14


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_k0_constant_strain_energy(seed):
    """For an affine field u = G x, u^T K0 u = h^3 (lam tr(eps)^2 + 2 mu eps:eps)."""
    rng = np.random.default_rng(seed)
    h, nu = 0.7, 0.3
    G = rng.standard_normal((3, 3))
    pos = np.array([[(a & 1) * h, ((a >> 1) & 1) * h, ((a >> 2) & 1) * h] for a in range(8)])
    u = (pos @ G.T).ravel()
    eps = 0.5 * (G + G.T)
    lam, mu = element.lame(1.0, nu)
    exact = h ** 3 * (lam * np.trace(eps) ** 2 + 2.0 * mu * np.sum(eps * eps))
    got = u @ element.k0(nu, h) @ u
    assert abs(got - exact) <= 1e-13 * abs(exact)


def test_k0_diagonal_closed_form():
    K = element.k0(0.3, 1.0)
    assert np.allclose(np.diag(K), 55.0 / 234.0, rtol=0, atol=1e-15)
    for nu in (0.1, 0.3, 0.4):
        for h in (1.0, 0.05):
            assert np.allclose(np.diag(element.k0(nu, h)), element.diag_entry(nu, h), rtol=1e-14, atol=0)
