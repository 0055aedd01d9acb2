"""Density filter, its adjoint, and the sensitivity filter (oracle, test
infrastructure only).

Sec. 2.1.3, Eq. 4: the sensitivity of element e is replaced by a weighted
average over the elements i whose centroids lie within R of e's centroid, with
the linearly decaying weight H_ei = max(0, R - ||x_e - x_i||) and the
density/volume factors rho_i / V_i (numerator) and rho_e / V_e (denominator).
The density filter, named in the same section as the alternative, averages the
densities themselves with weights H_ei V_i, normalised per element.

Readings (the paper is silent on them):
  * membership of N_e is strict (distance < R); H = 0 at distance R anyway;
  * at the domain boundary the stencil is truncated and each element is
    normalised by its own sum of weights (no padding);
  * the rho_e in Eq. 4's denominator is guarded as max(rho_e, 1e-3).

The functions below loop over element pairs by integer offset in plain
Python/NumPy; `*_bruteforce` loop over all element pairs by centroid distance
and exist to pin the offset form on tiny grids.
"""
import math
import numpy as np

from . import grid

SENS_GUARD = 1e-3


def stencil(r):
    """List of (dx, dy, dz, w) for integer offsets with distance < r,
    w = r - distance (in element units)."""
    m = int(math.ceil(r))
    out = []
    for dz in range(-m, m + 1):
        for dy in range(-m, m + 1):
            for dx in range(-m, m + 1):
                d = math.sqrt(dx * dx + dy * dy + dz * dz)
                if d < r:
                    out.append((dx, dy, dz, r - d))
    return out


def _shifted(field, nelx, nely, nelz, dx, dy, dz):
    """(values, valid) of field at element (i+dx, j+dy, k+dz) for every element."""
    f = np.asarray(field, dtype=np.float64).reshape(nelz, nely, nelx)
    out = np.zeros_like(f)
    valid = np.zeros(f.shape, dtype=bool)
    src = [slice(max(0, d), n + min(0, d)) for d, n in ((dz, nelz), (dy, nely), (dx, nelx))]
    dst = [slice(max(0, -d), n + min(0, -d)) for d, n in ((dz, nelz), (dy, nely), (dx, nelx))]
    out[tuple(dst)] = f[tuple(src)]
    valid[tuple(dst)] = True
    return out.ravel(), valid.ravel()


def weight_sums(nelx, nely, nelz, r):
    nel = nelx * nely * nelz
    s = np.zeros(nel)
    ones = np.ones(nel)
    for dx, dy, dz, w in stencil(r):
        _, valid = _shifted(ones, nelx, nely, nelz, dx, dy, dz)
        s += np.where(valid, w, 0.0)
    return s


def neighbour_counts(nelx, nely, nelz, r):
    nel = nelx * nely * nelz
    cnt = np.zeros(nel, dtype=np.int64)
    ones = np.ones(nel)
    for dx, dy, dz, _ in stencil(r):
        _, valid = _shifted(ones, nelx, nely, nelz, dx, dy, dz)
        cnt += valid
    return cnt


def density_filter(x, nelx, nely, nelz, r, h=1.0):
    """x~_e = sum_i H_ei V_i x_i / sum_i H_ei V_i."""
    V = h ** 3
    num = np.zeros(nelx * nely * nelz)
    den = np.zeros_like(num)
    for dx, dy, dz, w in stencil(r):
        v, valid = _shifted(x, nelx, nely, nelz, dx, dy, dz)
        num += np.where(valid, w * V * v, 0.0)
        den += np.where(valid, w * V, 0.0)
    return num / den


def density_filter_adjoint(g, nelx, nely, nelz, r, h=1.0):
    """Transpose of density_filter: dj = sum_e H_ej V_j g_e / sum_i H_ei V_i."""
    V = h ** 3
    den = weight_sums(nelx, nely, nelz, r) * V
    gs = np.asarray(g, dtype=np.float64) / den
    out = np.zeros_like(gs)
    for dx, dy, dz, w in stencil(r):
        v, valid = _shifted(gs, nelx, nely, nelz, dx, dy, dz)
        out += np.where(valid, w * V * v, 0.0)
    return out


def sensitivity_filter(x, dc, nelx, nely, nelz, r, h=1.0):
    """Eq. 4: dc~_e = sum_i (x_i/V_i) H_ei dc_i / ((max(x_e,g)/V_e) sum_i H_ei)."""
    V = h ** 3
    xdc = np.asarray(x, dtype=np.float64) / V * np.asarray(dc, dtype=np.float64)
    num = np.zeros(nelx * nely * nelz)
    den = np.zeros_like(num)
    for dx, dy, dz, w in stencil(r):
        v, valid = _shifted(xdc, nelx, nely, nelz, dx, dy, dz)
        num += np.where(valid, w * v, 0.0)
        den += np.where(valid, w, 0.0)
    xe = np.maximum(np.asarray(x, dtype=np.float64), SENS_GUARD) / V
    return num / (xe * den)


def _pair_weights_bruteforce(nelx, nely, nelz, r, h):
    c = grid.element_centroids(nelx, nely, nelz, h)
    d = np.sqrt(((c[:, None, :] - c[None, :, :]) ** 2).sum(-1))
    return np.where(d < r * h, r * h - d, 0.0) / h       # weights in element units


def density_filter_bruteforce(x, nelx, nely, nelz, r, h=1.0):
    H = _pair_weights_bruteforce(nelx, nely, nelz, r, h)
    V = h ** 3
    return (H * V) @ np.asarray(x, dtype=np.float64) / (H * V).sum(1)


def sensitivity_filter_bruteforce(x, dc, nelx, nely, nelz, r, h=1.0):
    H = _pair_weights_bruteforce(nelx, nely, nelz, r, h)
    V = h ** 3
    x = np.asarray(x, dtype=np.float64)
    return (H @ (x / V * dc)) / (np.maximum(x, SENS_GUARD) / V * H.sum(1))
