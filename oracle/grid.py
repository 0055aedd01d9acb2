"""Voxel grid numbering, boundary conditions and load vectors (oracle, test
infrastructure only).

The paper's state problem (Sec. 2.1.1, Eq. 2) is K(rho) U = F on a structured
hex mesh (Sec. 4.1).  The paper fixes no numbering; the reading used here is:

  node     n = i + (nelx+1) * (j + (nely+1) * k)
  element  e = i + nelx * (j + nely * k)        (lower corner at node (i,j,k))
  local    a = ax + 2*ay + 4*az                  (node (i+ax, j+ay, k+az))
  DOF      3*n + c,  c in {0:x, 1:y, 2:z}

z is the vertical axis (the paper's load is (0,0,-1), Sec. 4.2, and its MBB
"top" is z = 1, Sec. 4.3).

Built-in boundary conditions:

  CANTILEVER (0)  every DOF of every node on the x = 0 face is fixed; a total
                  downward load spread along the bottom edge (i = nelx, k = 0)
                  of the opposite face as the consistent nodal forces of a
                  uniform line load: end nodes carry half of an interior one.
  MBB (1)         half beam: u_x = 0 on x = 0 (symmetry), u_z = 0 on the
                  bottom-right edge (i = nelx, k = 0), u_y = 0 at node (0,0,0)
                  (removes the otherwise free y-translation; the load has no y
                  component, so the pin carries no reaction); the same line
                  load on the top edge at x = 0 (i = 0, k = nelz).
  CUSTOM (2)      mask and load supplied by the caller.

The paper's own variants (Sec. 4.2, 4.3: a 2 x 1 x 1 domain on 40 x 20 x 20
voxels), with the geometry scaled to the grid (Ly = nely h, Lz = nelz h,
r = min(Ly, Lz) / 10):

  CANTILEVER_CORNERS (3)  every DOF fixed on the x = 0 face nodes inside the
                  four corner squares 0.3 Ly x 0.3 Lz (y <= 0.3 Ly or
                  y >= 0.7 Ly, and likewise z); the load (0, 0, -1) on the
                  disc of radius r centred on the x = Lx face.
  MBB_STRIP (4)   u_x = 0 on x = 0 (symmetry); u_z = 0 on the bottom nodes of
                  the last element strip (k = 0, i >= nelx - 1: one element
                  wide); u_y = 0 at node (0,0,0) as for MBB; the load on the
                  half disc of radius r centred at (0, Ly/2, Lz) on the top
                  face.
  The loaded region is read as the boundary-face quads whose centroid lies in
  the disc (on grids too coarse for any, the quads nearest its centre), with
  a uniform traction: each tagged quad passes a quarter of its share to each
  of its four nodes, so a node carries -(load_total c) / (4 nq) in z, with c
  its tagged quads and nq their total.  All the geometric tests are integer
  arithmetic in half-element units.
"""
import numpy as np

BC_CANTILEVER, BC_MBB, BC_CUSTOM, BC_CANTILEVER_CORNERS, BC_MBB_STRIP = 0, 1, 2, 3, 4


def sizes(nelx, nely, nelz):
    nel = nelx * nely * nelz
    nn = (nelx + 1) * (nely + 1) * (nelz + 1)
    return nel, nn, 3 * nn


def node_index(nelx, nely, i, j, k):
    return i + (nelx + 1) * (j + (nely + 1) * k)


def element_nodes(nelx, nely, nelz):
    """(nel, 8) node indices; column a is local node a = ax + 2 ay + 4 az."""
    k, j, i = np.meshgrid(np.arange(nelz), np.arange(nely), np.arange(nelx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()          # element order e = i + nelx (j + nely k)
    cols = []
    for a in range(8):
        ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
        cols.append(node_index(nelx, nely, i + ax, j + ay, k + az))
    return np.stack(cols, axis=1).astype(np.int64)


def element_dofs(nelx, nely, nelz):
    """(nel, 24) DOF indices, ordered node-major: [3 n_0, 3 n_0 + 1, 3 n_0 + 2, 3 n_1, ...]."""
    en = element_nodes(nelx, nely, nelz)
    return (3 * en[:, :, None] + np.arange(3)[None, None, :]).reshape(en.shape[0], 24)


def node_coords(nelx, nely, nelz, h):
    """(nn, 3) coordinates of the nodes in node order."""
    k, j, i = np.meshgrid(np.arange(nelz + 1), np.arange(nely + 1), np.arange(nelx + 1), indexing="ij")
    return np.stack([i.ravel() * h, j.ravel() * h, k.ravel() * h], axis=1).astype(np.float64)


def element_centroids(nelx, nely, nelz, h):
    k, j, i = np.meshgrid(np.arange(nelz), np.arange(nely), np.arange(nelx), indexing="ij")
    return np.stack([(i.ravel() + 0.5) * h, (j.ravel() + 0.5) * h, (k.ravel() + 0.5) * h],
                    axis=1).astype(np.float64)


def _line_load_weight(nely, j):
    """Consistent nodal share of a unit uniform line load over nely segments:
    half a segment at each end, a whole one inside.  Returned as (w, nely) with
    the force -(load_total * w) / nely, so that both sides evaluate the same
    correctly rounded expression."""
    return 0.5 if (j == 0 or j == nely) else 1.0


def fixed_mask(nelx, nely, nelz, bc, custom_mask=None):
    """Boolean (ndof,) array, True = homogeneous Dirichlet DOF."""
    _, nn, ndof = sizes(nelx, nely, nelz)
    m = np.zeros(ndof, dtype=bool)
    if bc == BC_CUSTOM:
        cm = np.asarray(custom_mask).astype(bool).ravel()
        assert cm.size == ndof
        return cm.copy()
    if bc == BC_CANTILEVER:
        for k in range(nelz + 1):
            for j in range(nely + 1):
                n = node_index(nelx, nely, 0, j, k)
                m[3 * n:3 * n + 3] = True
        return m
    if bc == BC_MBB:
        for k in range(nelz + 1):
            for j in range(nely + 1):
                m[3 * node_index(nelx, nely, 0, j, k) + 0] = True
        for j in range(nely + 1):
            m[3 * node_index(nelx, nely, nelx, j, 0) + 2] = True
        m[3 * node_index(nelx, nely, 0, 0, 0) + 1] = True
        return m
    if bc == BC_CANTILEVER_CORNERS:
        for k in range(nelz + 1):
            for j in range(nely + 1):
                if _corner(j, nely) and _corner(k, nelz):
                    n = node_index(nelx, nely, 0, j, k)
                    m[3 * n:3 * n + 3] = True
        return m
    if bc == BC_MBB_STRIP:
        for k in range(nelz + 1):
            for j in range(nely + 1):
                m[3 * node_index(nelx, nely, 0, j, k) + 0] = True
        for i in (nelx - 1, nelx):
            for j in range(nely + 1):
                m[3 * node_index(nelx, nely, i, j, 0) + 2] = True
        m[3 * node_index(nelx, nely, 0, 0, 0) + 1] = True
        return m
    raise ValueError("unknown bc")


def _corner(j, n):
    """Node j of 0..n lies in a corner band: j h <= 0.3 L or j h >= 0.7 L."""
    return 10 * j <= 3 * n or 10 * j >= 7 * n


def loaded_quads(nelx, nely, nelz, bc):
    """Tagged boundary-face quads (a, b) of the disc (CANTILEVER_CORNERS: quad
    (j, k) of the x = Lx face) or half disc (MBB_STRIP: quad (i, j) of the
    z = Lz face).  4 d2 is the squared centroid distance to the centre in
    half-element units; a quad is tagged when 25 d2 <= min(nely, nelz)^2, or,
    when none is, when d2 is the smallest."""
    m = min(nely, nelz)
    if bc == BC_CANTILEVER_CORNERS:
        cells = [((2 * j + 1 - nely) ** 2 + (2 * k + 1 - nelz) ** 2, (j, k))
                 for k in range(nelz) for j in range(nely)]
    elif bc == BC_MBB_STRIP:
        cells = [((2 * i + 1) ** 2 + (2 * j + 1 - nely) ** 2, (i, j))
                 for j in range(nely) for i in range(nelx)]
    else:
        raise ValueError("bc without a loaded region")
    thr = m * m
    if not any(25 * d2 <= thr for d2, _ in cells):
        thr = 25 * min(d2 for d2, _ in cells)
    return [q for d2, q in cells if 25 * d2 <= thr]


def load_vector(nelx, nely, nelz, bc, load_total=1.0, custom_load=None):
    """(ndof,) float64 nodal force vector F."""
    _, nn, ndof = sizes(nelx, nely, nelz)
    f = np.zeros(ndof, dtype=np.float64)
    if bc == BC_CUSTOM:
        cl = np.asarray(custom_load, dtype=np.float64).ravel()
        assert cl.size == ndof
        return cl.copy()
    if bc in (BC_CANTILEVER_CORNERS, BC_MBB_STRIP):
        quads = loaded_quads(nelx, nely, nelz, bc)
        cnt = {}
        for a, b in quads:
            for da in (0, 1):
                for db in (0, 1):
                    if bc == BC_CANTILEVER_CORNERS:
                        n = node_index(nelx, nely, nelx, a + da, b + db)
                    else:
                        n = node_index(nelx, nely, a + da, b + db, nelz)
                    cnt[n] = cnt.get(n, 0) + 1
        for n, c in cnt.items():
            f[3 * n + 2] = -(load_total * c) / (4 * len(quads))
        return f
    if bc == BC_CANTILEVER:
        i, k = nelx, 0
    elif bc == BC_MBB:
        i, k = 0, nelz
    else:
        raise ValueError("unknown bc")
    for j in range(nely + 1):
        w = _line_load_weight(nely, j)
        f[3 * node_index(nelx, nely, i, j, k) + 2] = -(load_total * w) / nely
    return f
