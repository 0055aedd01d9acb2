"""Density -> signed distance transfer and ersatz volume fraction (oracle, test
infrastructure only).

  nodal_density_lsq   Sec. 3.2, Eqs. 25-27: per node, a linear least-squares
                      fit [1 x^T] a over the adjacent element centroids,
                      evaluated at the node; inverse-distance weights when the
                      fit is rank deficient (1 < m < 4, and -- a reading, the
                      paper is silent -- m >= 4 with coplanar centroids); copy
                      when m = 1.
  nodal_density_mean  On a voxel grid the map above is exactly the arithmetic
                      mean of the adjacent elements (interior: X^T X is
                      diagonal in centred coordinates; faces/edges: IDW with
                      equal distances; corners: copy).  This form fixes the
                      summation order (adjacent elements in increasing element
                      index, left-to-right adds, then times 1/m) so that the
                      inside/outside classification is reproducible bit for bit.
  marching_tets       Sec. 3.3: iso-surface at rho_t.  The paper uses
                      ParaView's Marching Cubes, whose tables are not in the
                      paper; the reading here is marching tetrahedra (which the
                      paper's software also supports) on the Kuhn six-tet split
                      of each voxel, which is watertight and has no ambiguous
                      cases.
  closest_point_dist  Sec. 3.4.1, Eq. 28: minimise ||x_n - x(lambda)||^2 over
                      the triangle; if the plane projection has all barycentric
                      coordinates >= 0 it is the answer, otherwise the minimum
                      lies on the boundary, i.e. on one of the three edges
                      (parameter clamped to [0, 1]).
  unsigned_distance   Eq. 29: minimum over all triangles (brute force).
  signed_distance     Eq. 30: phi = -d where rho_n >= rho_t, +d otherwise.
  volume_fraction     Sec. 4.1 ersatz: the solid (phi < 0) volume fraction of
                      each element for the piecewise-linear interpolant of phi
                      on the same Kuhn split, by clipping every tet and summing
                      sub-tet volumes.
"""
import itertools
import numpy as np

from . import grid

# Kuhn split: permutations of the axes in lexicographic order; tet for
# permutation p has corners v0 = 0, v1 = e_p0, v2 = e_p0 + e_p1, v3 = (1,1,1),
# written as local node numbers a = ax + 2 ay + 4 az.
PERMS = list(itertools.permutations(range(3)))


def kuhn_tets():
    tets = []
    for p in PERMS:
        v = [0, 0, 0]
        corners = [0]
        for axis in p:
            v[axis] = 1
            corners.append(v[0] + 2 * v[1] + 4 * v[2])
        tets.append(tuple(corners))
    return tets


KUHN = kuhn_tets()


# ---------------------------------------------------------------- Eqs. 25-27
def _adjacent_elements(nelx, nely, nelz, i, j, k):
    out = []
    for bz in (0, 1):
        for by in (0, 1):
            for bx in (0, 1):
                ei, ej, ek = i - 1 + bx, j - 1 + by, k - 1 + bz
                if 0 <= ei < nelx and 0 <= ej < nely and 0 <= ek < nelz:
                    out.append(ei + nelx * (ej + nely * ek))
    return out


def nodal_density_lsq(x, nelx, nely, nelz, h=1.0, coplanar_tol=1e-12):
    x = np.asarray(x, dtype=np.float64)
    cen = grid.element_centroids(nelx, nely, nelz, h)
    rho = np.zeros((nelx + 1) * (nely + 1) * (nelz + 1))
    for k in range(nelz + 1):
        for j in range(nely + 1):
            for i in range(nelx + 1):
                n = grid.node_index(nelx, nely, i, j, k)
                xn = np.array([i * h, j * h, k * h])
                adj = _adjacent_elements(nelx, nely, nelz, i, j, k)
                m = len(adj)
                if m == 1:
                    rho[n] = x[adj[0]]
                    continue
                X = np.hstack([np.ones((m, 1)), cen[adj]])
                full_rank = False
                if m >= 4:
                    sv = np.linalg.svd(X, compute_uv=False)
                    full_rank = sv[-1] > coplanar_tol * sv[0]
                if full_rank:
                    a = np.linalg.solve(X.T @ X, X.T @ x[adj])
                    rho[n] = np.array([1.0, *xn]) @ a
                else:
                    w = 1.0 / np.linalg.norm(cen[adj] - xn[None, :], axis=1)
                    rho[n] = (w @ x[adj]) / w.sum()
    return rho


def nodal_density_mean(x, nelx, nely, nelz):
    x = np.asarray(x, dtype=np.float64)
    rho = np.zeros((nelx + 1) * (nely + 1) * (nelz + 1))
    for k in range(nelz + 1):
        for j in range(nely + 1):
            for i in range(nelx + 1):
                adj = _adjacent_elements(nelx, nely, nelz, i, j, k)
                s = 0.0
                for e in adj:
                    s = s + x[e]
                rho[grid.node_index(nelx, nely, i, j, k)] = s * (1.0 / len(adj))
    return rho


# ---------------------------------------------------------------- Sec. 3.3
def _cut(pa, pb, ra, rb, rho_t):
    """Point where the linear interpolant crosses rho_t on edge a->b, a inside."""
    t = (rho_t - ra) / (rb - ra)
    return pa + t * (pb - pa)


def tet_triangles(P, R, rho_t):
    """Triangles of one tet: P (4,3) corner positions, R (4,) values."""
    ins = [r >= rho_t for r in R]
    I = [v for v in range(4) if ins[v]]
    O = [v for v in range(4) if not ins[v]]
    c = lambda a, b: _cut(P[a], P[b], R[a], R[b], rho_t)
    if len(I) == 1:
        a = I[0]
        return [(c(a, O[0]), c(a, O[1]), c(a, O[2]))]
    if len(I) == 3:
        d = O[0]
        return [(c(I[0], d), c(I[1], d), c(I[2], d))]
    if len(I) == 2:
        a, b = I
        cc, d = O
        pac, pad, pbd, pbc = c(a, cc), c(a, d), c(b, d), c(b, cc)
        return [(pac, pad, pbd), (pac, pbd, pbc)]
    return []


def marching_tets(rho_n, nelx, nely, nelz, h=1.0, rho_t=0.5):
    """Returns (triangles (nT,3,3), owner voxel (nT,), per-voxel count (nel,))."""
    rho_n = np.asarray(rho_n, dtype=np.float64)
    tris, owner = [], []
    counts = np.zeros(nelx * nely * nelz, dtype=np.int64)
    en = grid.element_nodes(nelx, nely, nelz)
    nc = grid.node_coords(nelx, nely, nelz, h)
    for e in range(en.shape[0]):
        vals = rho_n[en[e]]
        if np.all(vals >= rho_t) or np.all(vals < rho_t):
            continue
        pos = nc[en[e]]
        for tet in KUHN:
            for tr in tet_triangles(pos[list(tet)], vals[list(tet)], rho_t):
                tris.append(np.array(tr))
                owner.append(e)
                counts[e] += 1
    T = np.array(tris).reshape(-1, 3, 3)
    return T, np.array(owner, dtype=np.int64), counts


# ---------------------------------------------------------------- Eqs. 28-29
def _segment_dist2(x, a, b):
    ab = b - a
    L = ab @ ab
    t = 0.0 if L == 0.0 else min(1.0, max(0.0, ((x - a) @ ab) / L))
    p = a + t * ab
    return (x - p) @ (x - p)


def closest_point_dist2(x, tri):
    """Squared distance from x to the triangle tri (3,3)."""
    q1, q2, q3 = tri
    e1, e2 = q2 - q1, q3 - q1
    G = np.array([[e1 @ e1, e1 @ e2], [e1 @ e2, e2 @ e2]])
    det = G[0, 0] * G[1, 1] - G[0, 1] ** 2
    if det > 1e-30 * (G[0, 0] * G[1, 1] + 1e-300):
        rhs = np.array([(x - q1) @ e1, (x - q1) @ e2])
        l2, l3 = np.linalg.solve(G, rhs)
        l1 = 1.0 - l2 - l3
        if l1 >= 0.0 and l2 >= 0.0 and l3 >= 0.0:
            p = q1 + l2 * e1 + l3 * e2
            return (x - p) @ (x - p)
    return min(_segment_dist2(x, q1, q2), _segment_dist2(x, q2, q3), _segment_dist2(x, q3, q1))


def unsigned_distance(points, T):
    """Eq. 29 by brute force over all triangles."""
    d = np.full(len(points), np.inf)
    for n, xpt in enumerate(points):
        best = np.inf
        for tri in T:
            best = min(best, closest_point_dist2(xpt, tri))
        d[n] = np.sqrt(best)
    return d


def unsigned_distance_vec(points, T):
    """Same minimum as unsigned_distance, vectorised over triangles (same
    case rule: plane projection if inside, else the nearest of the three
    clamped edge projections)."""
    points = np.asarray(points, dtype=np.float64)
    if len(T) == 0:
        return np.full(len(points), np.inf)
    q1, q2, q3 = T[:, 0], T[:, 1], T[:, 2]
    e1, e2 = q2 - q1, q3 - q1
    g11 = (e1 * e1).sum(1)
    g12 = (e1 * e2).sum(1)
    g22 = (e2 * e2).sum(1)
    det = g11 * g22 - g12 * g12
    ok = det > 1e-30 * (g11 * g22 + 1e-300)

    def seg(xp, a, b):
        ab = b - a
        L = (ab * ab).sum(1)
        t = np.where(L > 0, ((xp - a) * ab).sum(1) / np.where(L > 0, L, 1.0), 0.0)
        t = np.clip(t, 0.0, 1.0)
        p = a + t[:, None] * ab
        return ((xp - p) ** 2).sum(1)

    out = np.empty(len(points))
    for n, xp in enumerate(points):
        w = xp[None, :] - q1
        r1 = (w * e1).sum(1)
        r2 = (w * e2).sum(1)
        sdet = np.where(ok, det, 1.0)
        l2 = (g22 * r1 - g12 * r2) / sdet
        l3 = (g11 * r2 - g12 * r1) / sdet
        l1 = 1.0 - l2 - l3
        inside = ok & (l1 >= 0) & (l2 >= 0) & (l3 >= 0)
        p = q1 + l2[:, None] * e1 + l3[:, None] * e2
        dplane = ((xp[None, :] - p) ** 2).sum(1)
        dedge = np.minimum(np.minimum(seg(xp, q1, q2), seg(xp, q2, q3)), seg(xp, q3, q1))
        out[n] = np.sqrt(np.min(np.where(inside, dplane, dedge)))
    return out


def signed_distance(d, rho_n, rho_t=0.5):
    """Eq. 30."""
    return np.where(np.asarray(rho_n) >= rho_t, -d, d)


# ---------------------------------------------------------------- ersatz vf
def _tet_volume(a, b, c, d):
    return abs(np.linalg.det(np.array([b - a, c - a, d - a]))) / 6.0


def tet_negative_fraction(P, F):
    """Fraction of tet P (4,3) where the linear interpolant of F (4,) is < 0,
    by clipping the tet with the plane F = 0 and summing sub-tet volumes."""
    V = _tet_volume(*P)
    neg = [v for v in range(4) if F[v] < 0.0]
    pos = [v for v in range(4) if F[v] >= 0.0]
    if len(neg) == 0:
        return 0.0
    if len(neg) == 4:
        return 1.0

    def cut(a, b):   # F[a] < 0 <= F[b]
        t = F[a] / (F[a] - F[b])
        return P[a] + t * (P[b] - P[a])

    if len(neg) == 1:
        a = neg[0]
        return _tet_volume(P[a], cut(a, pos[0]), cut(a, pos[1]), cut(a, pos[2])) / V
    if len(neg) == 3:
        d = pos[0]
        small = _tet_volume(P[d], cut(neg[0], d), cut(neg[1], d), cut(neg[2], d))
        return (V - small) / V
    a, b = neg
    c, d = pos
    A = (P[a], cut(a, c), cut(a, d))
    B = (P[b], cut(b, c), cut(b, d))
    vol = (_tet_volume(A[0], A[1], A[2], B[0]) + _tet_volume(A[1], A[2], B[0], B[1])
           + _tet_volume(A[2], B[0], B[1], B[2]))
    return vol / V


def volume_fraction(phi, nelx, nely, nelz, h=1.0):
    phi = np.asarray(phi, dtype=np.float64)
    en = grid.element_nodes(nelx, nely, nelz)
    nc = grid.node_coords(nelx, nely, nelz, h)
    vf = np.zeros(en.shape[0])
    for e in range(en.shape[0]):
        vals = phi[en[e]]
        if np.all(vals < 0.0):
            vf[e] = 1.0
            continue
        if np.all(vals >= 0.0):
            continue
        pos = nc[en[e]]
        acc = 0.0
        for tet in KUHN:
            acc += tet_negative_fraction(pos[list(tet)], vals[list(tet)])
        vf[e] = acc / 6.0
    return vf


def density_to_sdf(x, nelx, nely, nelz, h=1.0, rho_t=0.5, vectorised=True):
    """Full transfer: (phi, rho_n, vf, triangles, counts)."""
    rho_n = nodal_density_mean(x, nelx, nely, nelz)
    T, owner, counts = marching_tets(rho_n, nelx, nely, nelz, h, rho_t)
    pts = grid.node_coords(nelx, nely, nelz, h)
    d = unsigned_distance_vec(pts, T) if vectorised else unsigned_distance(pts, T)
    phi = signed_distance(d, rho_n, rho_t)
    vf = volume_fraction(phi, nelx, nely, nelz, h)
    return phi, rho_n, vf, T, counts
