"""Assembled-K state solve, compliance and sensitivity (oracle, test
infrastructure only).

  modulus            Eq. 1   E_e = Emin + x_e^p (E0 - Emin)
  assemble           Eq. 2   K = sum_e E_e k_e^0 on the element->DOF map (CSR)
  apply_masked               the library's operator: y = K u with the fixed DOFs
                             zeroed on input and identity rows on output
  solve_direct       Eq. 2   K_ff u_f = f_f by sparse LU, u_fixed = 0
  solve_pcg          Eq. 2   the same by Jacobi-preconditioned CG in float64
  compliance         Eq. 2   c = f^T u (= u^T K u at the solution)
  element_energy     Eq. 3   s_e = u_e^T k_e^0 u_e
  sensitivity        Eq. 3   dc_e = -p x_e^(p-1) (E0 - Emin) s_e
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import grid
from . import element


def modulus(x, E0, Emin, penal):
    x = np.asarray(x, dtype=np.float64)
    return Emin + x ** penal * (E0 - Emin)


def assemble(nelx, nely, nelz, E, K0):
    """CSR ndof x ndof global stiffness K = sum_e E_e K0 (duplicates summed)."""
    edof = grid.element_dofs(nelx, nely, nelz)
    nel = edof.shape[0]
    _, _, ndof = grid.sizes(nelx, nely, nelz)
    rows = np.repeat(edof, 24, axis=1).ravel()
    cols = np.tile(edof, (1, 24)).ravel()
    vals = (np.asarray(E, dtype=np.float64)[:, None] * K0.ravel()[None, :]).ravel()
    K = sp.coo_matrix((vals, (rows, cols)), shape=(ndof, ndof)).tocsr()
    K.sum_duplicates()
    return K


def apply_masked(K, fixed, u):
    """y = K u_free, with y_fixed = u_fixed (identity rows/cols on fixed DOFs)."""
    u = np.asarray(u, dtype=np.float64)
    u0 = u.copy()
    u0[fixed] = 0.0
    y = K @ u0
    y[fixed] = u[fixed]
    return y


def solve_direct(K, f, fixed):
    free = np.flatnonzero(~fixed)
    Kff = K[free][:, free].tocsc()
    u = np.zeros(K.shape[0])
    u[free] = spla.spsolve(Kff, f[free])
    return u


def solve_pcg(K, f, fixed, rtol=1e-10, maxit=100000, u0=None):
    """Jacobi-PCG on the reduced system K_ff u_f = f_f.  Stops when the true
    residual ||f_f - K_ff u_f||_2 / ||f_f||_2 <= rtol (checked whenever the
    recursive residual says so).  Returns (u, iterations, rel_res)."""
    free = np.flatnonzero(~fixed)
    Kff = K[free][:, free].tocsr()
    b = f[free]
    nb = np.linalg.norm(b)
    x = np.zeros(free.size) if u0 is None else np.asarray(u0, dtype=np.float64)[free].copy()
    dinv = 1.0 / Kff.diagonal()
    r = b - Kff @ x
    if nb == 0.0:
        u = np.zeros(K.shape[0])
        return u, 0, 0.0
    z = dinv * r
    p = z.copy()
    rz = r @ z
    it = 0
    rel = np.linalg.norm(r) / nb
    while rel > rtol and it < maxit:
        q = Kff @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        rel = np.linalg.norm(r) / nb
        if rel <= rtol:
            r_true = b - Kff @ x
            rel = np.linalg.norm(r_true) / nb
            if rel <= rtol:
                break
            r = r_true
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    u = np.zeros(K.shape[0])
    u[free] = x
    return u, it, rel


def compliance(f, u):
    return float(np.dot(f, u))


def element_energy(nelx, nely, nelz, K0, u):
    """s_e = u_e^T K0 u_e for every element."""
    ue = np.asarray(u, dtype=np.float64)[grid.element_dofs(nelx, nely, nelz)]
    return np.einsum("ei,ij,ej->e", ue, K0, ue)


def sensitivity(x, s, E0, Emin, penal):
    x = np.asarray(x, dtype=np.float64)
    return -penal * x ** (penal - 1.0) * (E0 - Emin) * s


def problem_arrays(nelx, nely, nelz, bc, load_total=1.0, custom_mask=None, custom_load=None):
    fixed = grid.fixed_mask(nelx, nely, nelz, bc, custom_mask)
    f = grid.load_vector(nelx, nely, nelz, bc, load_total, custom_load)
    f = np.where(fixed, 0.0, f)
    return fixed, f


def full_solve(nelx, nely, nelz, x, *, h=1.0, E0=1.0, Emin=1e-9, nu=0.3, penal=3.0,
               bc=grid.BC_CANTILEVER, load_total=1.0, method="direct", rtol=1e-12):
    """Convenience: (u, c, dc, info) for one design."""
    K0 = element.k0(nu, h)
    E = modulus(x, E0, Emin, penal)
    K = assemble(nelx, nely, nelz, E, K0)
    fixed, f = problem_arrays(nelx, nely, nelz, bc, load_total)
    if method == "direct":
        u = solve_direct(K, f, fixed)
        info = {"iters": 0}
    else:
        u, it, rel = solve_pcg(K, f, fixed, rtol=rtol)
        info = {"iters": it, "rel_res": rel}
    s = element_energy(nelx, nely, nelz, K0, u)
    dc = sensitivity(x, s, E0, Emin, penal)
    return u, compliance(f, u), dc, info


def apply_rows(nelx, nely, nelz, E, K0, u, fixed, nodes):
    """Rows of the masked operator at the given nodes, straight from the
    definition y_n = sum over the elements e around n of E_e (K0 u_e)[node n]
    (fixed DOFs zero on input, identity rows on output).  Returns (len(nodes), 3).
    Used to check the operator on grids too large to assemble."""
    u = np.asarray(u, dtype=np.float64)
    u0 = np.where(fixed, 0.0, u)
    out = np.zeros((len(nodes), 3))
    NX, NY = nelx + 1, nely + 1
    for r, n in enumerate(nodes):
        i, j, k = n % NX, (n // NX) % NY, n // (NX * NY)
        acc = np.zeros(3)
        for bz in (0, 1):
            for by in (0, 1):
                for bx in (0, 1):
                    ei, ej, ek = i - 1 + bx, j - 1 + by, k - 1 + bz
                    if not (0 <= ei < nelx and 0 <= ej < nely and 0 <= ek < nelz):
                        continue
                    e = ei + nelx * (ej + nely * ek)
                    a = (1 - bx) + 2 * (1 - by) + 4 * (1 - bz)     # corner of e at node n
                    dofs = []
                    for b in range(8):
                        nb = grid.node_index(nelx, nely, ei + (b & 1), ej + ((b >> 1) & 1), ek + (b >> 2))
                        dofs.extend([3 * nb, 3 * nb + 1, 3 * nb + 2])
                    acc += E[e] * (K0[3 * a:3 * a + 3, :] @ u0[dofs])
        for c in range(3):
            out[r, c] = u[3 * n + c] if fixed[3 * n + c] else acc[c]
    return out
