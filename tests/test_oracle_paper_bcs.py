"""Pins for the paper's own boundary-condition variants (Sec. 4.2: cantilever
on four corner supports with a disc load; Sec. 4.3: MBB with a one-element
support strip and a half-disc load), on its 40 x 20 x 20 grid of a 2 x 1 x 1
domain (h = 0.05).

  * counts by hand: four 7 x 7-node corner squares (j h <= 0.3 or >= 0.7);
    the MBB's x = 0 face (u_x), two node rows of the strip (u_z) and the
    y-pin; the disc of radius 2 elements about a node tags the 12 quads whose
    centroid offsets are (+-1, +-1), (+-1, +-3), (+-3, +-1) half-elements, the
    half disc the 6 quads (1, +-1), (3, +-1), (1, +-3);
  * the nodal loads are z-only and sum to the total;
  * the reactions balance the load (K non-singular: the supports remove every
    rigid mode);
  * dc is mirror-symmetric in y (both) and in z (corner cantilever: the
    mirror flips only the load's sign)."""
import numpy as np
import pytest

from oracle import element, fem, grid


def test_counts_and_load():
    m3 = grid.fixed_mask(40, 20, 20, grid.BC_CANTILEVER_CORNERS)
    assert m3.sum() == 4 * 7 * 7 * 3
    m4 = grid.fixed_mask(40, 20, 20, grid.BC_MBB_STRIP)
    assert m4.sum() == 21 * 21 + 2 * 21 + 1
    q3 = grid.loaded_quads(40, 20, 20, grid.BC_CANTILEVER_CORNERS)
    off = sorted((2 * j + 1 - 20, 2 * k + 1 - 20) for j, k in q3)
    want = sorted({(a, b) for a in (-3, -1, 1, 3) for b in (-3, -1, 1, 3)
                   if not (abs(a) == 3 and abs(b) == 3)})
    assert off == want
    q4 = grid.loaded_quads(40, 20, 20, grid.BC_MBB_STRIP)
    assert sorted((2 * i + 1, 2 * j + 1 - 20) for i, j in q4) == sorted(
        [(1, -1), (1, 1), (3, -1), (3, 1), (1, -3), (1, 3)])
    for bc in (grid.BC_CANTILEVER_CORNERS, grid.BC_MBB_STRIP):
        f = grid.load_vector(40, 20, 20, bc, load_total=1.0).reshape(-1, 3)
        assert np.all(f[:, :2] == 0.0) and abs(f[:, 2].sum() + 1.0) < 1e-15
        # a node shared by four tagged quads carries four quarters
        assert np.isclose(f[:, 2].min(), -4.0 / (4 * (12 if bc == 3 else 6)))
    # coarse grids still get a loaded region
    assert len(grid.loaded_quads(3, 2, 2, grid.BC_CANTILEVER_CORNERS)) == 4
    assert len(grid.loaded_quads(5, 4, 3, grid.BC_MBB_STRIP)) == 2


@pytest.mark.parametrize("bc", [grid.BC_CANTILEVER_CORNERS, grid.BC_MBB_STRIP])
def test_equilibrium_and_symmetry(bc):
    nelx, nely, nelz, h = 20, 10, 10, 0.1
    x = np.full(nelx * nely * nelz, 0.4)
    u, c, dc, _ = fem.full_solve(nelx, nely, nelz, x, h=h, bc=bc)
    K0 = element.k0(0.3, h)
    K = fem.assemble(nelx, nely, nelz, fem.modulus(x, 1.0, 1e-9, 3.0), K0)
    fixed, f = fem.problem_arrays(nelx, nely, nelz, bc)
    reac = (K @ u)[fixed]
    r = np.zeros(u.size)
    r[fixed] = reac
    r = r.reshape(-1, 3).sum(axis=0)
    assert np.max(np.abs(r + f.reshape(-1, 3).sum(axis=0))) < 1e-9
    assert c > 0.0 and np.all(dc <= 0.0)
    g = dc.reshape(nelz, nely, nelx)
    assert np.max(np.abs(g - g[:, ::-1, :])) < 1e-9 * np.abs(g).max()
    if bc == grid.BC_CANTILEVER_CORNERS:
        assert np.max(np.abs(g - g[::-1, :, :])) < 1e-9 * np.abs(g).max()


def test_oracle_simp_matches_paper_iteration_counts():
    """The oracle's SIMP loop on the two problems, stopped at Delta rho_max =
    8 % and 4 %, takes the iteration counts the paper prints in its tables
    (Secs. 4.2-4.3), to within two.  The oracle's run takes about ten minutes
    per case on one core, so it is stored: tests/golden/make_paper_simp.py
    (which calls only the oracle) wrote paper_simp_oracle.json."""
    import json
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    table = json.load(open(os.path.join(here, "paper_simp_table.json")))
    orc = json.load(open(os.path.join(here, "paper_simp_oracle.json")))
    for name in ("cantilever_corners", "mbb_strip"):
        paper = dict(zip(table["delta_rho_max"], table[name]["iterations"]))
        for tol in (0.08, 0.04):
            rec = orc[name][str(tol)]
            assert abs(rec["iterations"] - paper[tol]) <= 2, (name, tol)
            assert rec["change"][-1] <= tol < rec["change"][-2]
            assert all(abs(v / 0.4 - 1.0) <= 1.5e-3 for v in rec["volume"])
