"""Level-set evolution and reinitialisation on the node grid (oracle, test
infrastructure only).

Sec. 2.2.7 evolves phi by the Hamilton-Jacobi equation phi_t + v |grad phi| = 0
(Eq. 21) with forward Euler in time and the first-order Godunov upwind stencil
in space, for a fixed number of steps with dt = gamma h / max|v| (the CFL bound
of Eq. 22 scaled by a CFL number gamma in (0, 1)).  Sec. 2.2.8 restores the
distance property by solving phi_t + S(phi) (|grad phi| - 1) = 0 (Eq. 23) with
the same scheme, the smeared sign S(phi) = phi / sqrt(phi^2 + h^2 |grad phi|^2)
(Eq. 24) recomputed from the current phi at every pseudo-step, until the
largest change of a pseudo-step falls below a tolerance.

phi and v live on the (nelx+1)(nely+1)(nelz+1) nodes, index
n = i + NX (j + NY k), spacing h.  Readings where the paper is silent:

  * one-sided differences  D-x = (phi_i - phi_{i-1}) / h,
                           D+x = (phi_{i+1} - phi_i) / h  (likewise y, z);
    at the box faces the missing neighbour is the node itself (homogeneous
    Neumann), so the difference across the face is 0;
  * Godunov upwind magnitudes for a speed of either sign:
        g+ = sqrt(sum over axes of max(D-, 0)^2 + min(D+, 0)^2)   (speed > 0)
        g- = sqrt(sum over axes of min(D-, 0)^2 + max(D+, 0)^2)   (speed < 0)
    summed x, then y, then z;
  * evolution:      phi <- phi - dt (max(v, 0) g+ + min(v, 0) g-),
                    dt = gamma h / max|v| (no motion when v = 0 everywhere);
  * reinitialisation: phi <- phi - dtau (max(S, 0)(g+ - 1) + min(S, 0)(g- - 1))
    with dtau = gamma h (|S| <= 1), |grad phi| inside S from central
    differences (phi_{i+1} - phi_{i-1}) / (2h) with the same face rule, and
    S = 0 where phi^2 + h^2 |grad phi|^2 = 0;
  * the reinitialisation stops after the first pseudo-step whose largest
    |change| is < tol; reaching max_steps first is an error.

  godunov_magnitudes   (g+, g-) of a node field
  advect               n steps of Eq. 21 with the Eq. 22 step
  reinit_step          one pseudo-step of Eq. 23 with Eq. 24
  reinit               pseudo-steps to the stop rule
"""
import numpy as np


def _grid(phi, nelx, nely, nelz):
    return np.asarray(phi, dtype=np.float64).reshape(nelz + 1, nely + 1, nelx + 1)


def _neighbours(p):
    """(minus, plus) neighbour values along x, y, z with the face rule."""
    out = []
    for ax in (2, 1, 0):                       # x, y, z on the (k, j, i) array
        m = np.concatenate([np.take(p, [0], axis=ax), np.delete(p, -1, axis=ax)], axis=ax)
        q = np.concatenate([np.delete(p, 0, axis=ax), np.take(p, [-1], axis=ax)], axis=ax)
        out.append((m, q))
    return out


def godunov_magnitudes(phi, nelx, nely, nelz, h):
    p = _grid(phi, nelx, nely, nelz)
    sp = np.zeros_like(p)
    sm = np.zeros_like(p)
    for m, q in _neighbours(p):
        dm = (p - m) / h
        dq = (q - p) / h
        sp = sp + np.maximum(dm, 0.0) ** 2 + np.minimum(dq, 0.0) ** 2
        sm = sm + np.minimum(dm, 0.0) ** 2 + np.maximum(dq, 0.0) ** 2
    return np.sqrt(sp).ravel(), np.sqrt(sm).ravel()


def cfl_step(v, gamma, h):
    vmax = float(np.max(np.abs(v)))
    return 0.0 if vmax == 0.0 else gamma * h / vmax


def advect(phi, v, nelx, nely, nelz, h=1.0, gamma=0.5, nsteps=1):
    """Returns (phi after nsteps, dt)."""
    phi = np.array(phi, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    if not (np.all(np.isfinite(phi)) and np.all(np.isfinite(v))):
        raise ValueError("non-finite phi or v")
    dt = cfl_step(v, gamma, h)
    for _ in range(nsteps):
        gp, gm = godunov_magnitudes(phi, nelx, nely, nelz, h)
        phi = phi - dt * (np.maximum(v, 0.0) * gp + np.minimum(v, 0.0) * gm)
    return phi, dt


def smeared_sign(phi, nelx, nely, nelz, h):
    p = _grid(phi, nelx, nely, nelz)
    g2 = np.zeros_like(p)
    for m, q in _neighbours(p):
        d = (q - m) / (2.0 * h)
        g2 = g2 + d * d
    den = np.sqrt(p * p + h * h * g2)
    s = np.divide(p, den, out=np.zeros_like(p), where=den > 0.0)
    return s.ravel()


def reinit_step(phi, nelx, nely, nelz, h, dtau):
    s = smeared_sign(phi, nelx, nely, nelz, h)
    gp, gm = godunov_magnitudes(phi, nelx, nely, nelz, h)
    return phi - dtau * (np.maximum(s, 0.0) * (gp - 1.0) + np.minimum(s, 0.0) * (gm - 1.0))


def reinit(phi, nelx, nely, nelz, h=1.0, gamma=0.5, tol=1e-6, max_steps=1000):
    """Returns (phi, steps, last max |change|); raises RuntimeError when
    max_steps pass without a change below tol."""
    phi = np.array(phi, dtype=np.float64)
    if not np.all(np.isfinite(phi)):
        raise ValueError("non-finite phi")
    dtau = gamma * h
    for step in range(1, max_steps + 1):
        new = reinit_step(phi, nelx, nely, nelz, h, dtau)
        change = float(np.max(np.abs(new - phi)))
        phi = new
        if change < tol:
            return phi, step, change
    raise RuntimeError("reinitialisation: change still >= tol after %d steps" % max_steps)
