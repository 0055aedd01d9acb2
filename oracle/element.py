"""Unit-modulus hex8 element stiffness k_e^0 (oracle, test infrastructure only).

Sec. 2.1.2 (Eq. 3) defines k_e^0 as the element stiffness for unit Young's
modulus; Eq. 2 assembles K = sum_e E_e k_e^0 with E_e from Eq. 1.  The paper
does not state the element or its quadrature (it uses Gridap, Sec. 4.1).  The
reading here is the standard fully integrated trilinear hexahedron on the cube
[0,h]^3, isotropic linear elasticity, Voigt strains with engineering shear,
integrated by 2x2x2 Gauss (exact on a cube: every integrand has degree <= 2 in
each variable).
"""
import numpy as np


def lame(E, nu):
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def constitutive(E, nu):
    """6x6 isotropic D in Voigt order (xx, yy, zz, yz, xz, xy), engineering shear."""
    lam, mu = lame(E, nu)
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[0, 0] = D[1, 1] = D[2, 2] = lam + 2.0 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    return D


def shape_gradients(xi, eta, zeta, h):
    """(8, 3) physical gradients of the trilinear shape functions at the
    reference point (xi, eta, zeta) in [0,1]^3; local node a = ax + 2 ay + 4 az."""
    g = np.zeros((8, 3))
    r = (xi, eta, zeta)
    for a in range(8):
        bits = (a & 1, (a >> 1) & 1, (a >> 2) & 1)
        f = [r[d] if bits[d] else 1.0 - r[d] for d in range(3)]
        df = [1.0 if bits[d] else -1.0 for d in range(3)]
        g[a, 0] = df[0] * f[1] * f[2] / h
        g[a, 1] = f[0] * df[1] * f[2] / h
        g[a, 2] = f[0] * f[1] * df[2] / h
    return g


def strain_matrix(grads):
    """6x24 B with strain = B u_e, u_e ordered [u0x u0y u0z u1x ...]."""
    B = np.zeros((6, 24))
    for a in range(8):
        gx, gy, gz = grads[a]
        c = 3 * a
        B[0, c + 0] = gx
        B[1, c + 1] = gy
        B[2, c + 2] = gz
        B[3, c + 1] = gz
        B[3, c + 2] = gy
        B[4, c + 0] = gz
        B[4, c + 2] = gx
        B[5, c + 0] = gy
        B[5, c + 1] = gx
    return B


def k0(nu=0.3, h=1.0, order=2):
    """24x24 unit-modulus element stiffness by order x order x order Gauss."""
    pts, wts = np.polynomial.legendre.leggauss(order)
    pts = 0.5 * (pts + 1.0)          # map to [0, 1]
    wts = 0.5 * wts
    D = constitutive(1.0, nu)
    K = np.zeros((24, 24))
    for a, wa in zip(pts, wts):
        for b, wb in zip(pts, wts):
            for c, wc in zip(pts, wts):
                B = strain_matrix(shape_gradients(a, b, c, h))
                K += (wa * wb * wc * h ** 3) * (B.T @ D @ B)
    return 0.5 * (K + K.T)


def diag_entry(nu=0.3, h=1.0):
    """Every diagonal entry of k_e^0 on a cube equals h (lam + 4 mu) / 9 (unit E):
    the (c,c) entry of node a integrates (lam+2mu) (d_c N_a)^2 + mu sum_{d!=c}
    (d_d N_a)^2, and each integral of (d_d N_a)^2 over the cube is h/9."""
    lam, mu = lame(1.0, nu)
    return h * (lam + 4.0 * mu) / 9.0
