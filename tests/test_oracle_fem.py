"""Pins for the oracle's state solve, compliance and sensitivity (Eqs. 1-3).

Independent checks: a closed-form uniaxial-tension solution, the patch test,
equilibrium of reactions, direct vs iterative solve, the compliance identity
f^T u = u^T K u = sum_e E_e s_e, and central finite differences of the
compliance for Eq. 3.
"""
import numpy as np
import pytest

from oracle import element, fem, grid


def _tension_problem(nelx, nely, nelz, h, t, nu):
    """Symmetry planes x=0 (u_x), y=0 (u_y), z=0 (u_z) and a uniform traction t
    on x = nelx*h, as consistent nodal forces (face corners 1/4, face edges 1/2,
    face interior 1, times t h^2)."""
    _, nn, ndof = grid.sizes(nelx, nely, nelz)
    mask = np.zeros(ndof, dtype=bool)
    load = np.zeros(ndof)
    for k in range(nelz + 1):
        for j in range(nely + 1):
            for i in range(nelx + 1):
                n = grid.node_index(nelx, nely, i, j, k)
                if i == 0:
                    mask[3 * n] = True
                if j == 0:
                    mask[3 * n + 1] = True
                if k == 0:
                    mask[3 * n + 2] = True
                if i == nelx:
                    wy = 0.5 if j in (0, nely) else 1.0
                    wz = 0.5 if k in (0, nelz) else 1.0
                    load[3 * n] = t * h * h * wy * wz
    return mask, load


def test_uniaxial_tension_closed_form():
    nelx, nely, nelz, h, t, nu, E0 = 5, 3, 4, 0.5, 2.0, 0.3, 3.0
    mask, load = _tension_problem(nelx, nely, nelz, h, t, nu)
    K0 = element.k0(nu, h)
    E = np.full(nelx * nely * nelz, E0)
    K = fem.assemble(nelx, nely, nelz, E, K0)
    u = fem.solve_direct(K, load, mask).reshape(-1, 3)
    X = grid.node_coords(nelx, nely, nelz, h)
    exact = np.stack([t / E0 * X[:, 0], -nu * t / E0 * X[:, 1], -nu * t / E0 * X[:, 2]], axis=1)
    assert np.max(np.abs(u - exact)) < 1e-12
    L, A = nelx * h, nely * h * nelz * h
    assert abs(fem.compliance(load, u.ravel()) - t * t * A * L / E0) < 1e-12


def test_patch_test_interior_reproduces_affine_field():
    rng = np.random.default_rng(3)
    nelx, nely, nelz, h = 4, 3, 3, 1.0
    G = rng.standard_normal((3, 3))
    tr = rng.standard_normal(3)
    X = grid.node_coords(nelx, nely, nelz, h)
    uex = (X @ G.T + tr).ravel()
    K = fem.assemble(nelx, nely, nelz, np.full(nelx * nely * nelz, 1.7), element.k0(0.3, h))
    bnd = np.zeros(len(X), dtype=bool)
    bnd |= (X[:, 0] == 0) | (X[:, 0] == nelx * h) | (X[:, 1] == 0) | (X[:, 1] == nely * h)
    bnd |= (X[:, 2] == 0) | (X[:, 2] == nelz * h)
    fixed = np.repeat(bnd, 3)
    free = np.flatnonzero(~fixed)
    fx = np.flatnonzero(fixed)
    Kff = K[free][:, free].tocsc()
    import scipy.sparse.linalg as spla
    ui = spla.spsolve(Kff, -(K[free][:, fx] @ uex[fx]))
    assert np.max(np.abs(ui - uex[free])) < 1e-12


@pytest.fixture(scope="module")
def config0():
    nelx, nely, nelz = 24, 12, 6
    x = np.full(nelx * nely * nelz, 0.5)
    K0 = element.k0(0.3, 1.0)
    E = fem.modulus(x, 1.0, 1e-9, 3.0)
    K = fem.assemble(nelx, nely, nelz, E, K0)
    fixed, f = fem.problem_arrays(nelx, nely, nelz, grid.BC_CANTILEVER)
    u = fem.solve_direct(K, f, fixed)
    return dict(nelx=nelx, nely=nely, nelz=nelz, x=x, K0=K0, E=E, K=K, fixed=fixed, f=f, u=u)


def test_config0_equilibrium_and_compliance_identity(config0):
    c = config0
    Ku = c["K"] @ c["u"]
    react = Ku[c["fixed"]].reshape(-1, 3) if c["fixed"].sum() % 3 == 0 else None
    # reactions at the fixed DOFs balance the applied load, per component
    for comp in range(3):
        sel = np.zeros_like(c["fixed"])
        sel[comp::3] = True
        R = Ku[c["fixed"] & sel].sum()
        F = c["f"][~c["fixed"] & sel].sum()
        assert abs(R + F) < 1e-9
    assert react is not None
    comp_fu = fem.compliance(c["f"], c["u"])
    comp_uku = c["u"] @ (c["K"] @ c["u"])
    s = fem.element_energy(c["nelx"], c["nely"], c["nelz"], c["K0"], c["u"])
    comp_es = float(np.sum(c["E"] * s))
    assert abs(comp_fu - comp_uku) < 1e-9 * comp_fu
    assert abs(comp_fu - comp_es) < 1e-9 * comp_fu
    # value from an independent scratch implementation under the same readings
    # (z vertical, consistent line-load shares); a consistency check only
    assert abs(comp_fu - 172.660276420466) < 1e-8


def test_config0_pcg_matches_direct(config0):
    c = config0
    u, it, rel = fem.solve_pcg(c["K"], c["f"], c["fixed"], rtol=1e-10)
    assert rel <= 1e-10
    assert np.linalg.norm(u - c["u"]) <= 1e-8 * np.linalg.norm(c["u"])
    assert 100 < it < 1000


def test_config0_mirror_symmetry(config0):
    c = config0
    s = fem.element_energy(c["nelx"], c["nely"], c["nelz"], c["K0"], c["u"]).reshape(6, 12, 24)
    assert np.allclose(s, s[:, ::-1, :], rtol=1e-9, atol=1e-10 * s.max())


def test_apply_masked_identity_rows(config0):
    c = config0
    rng = np.random.default_rng(0)
    v = rng.standard_normal(c["f"].size)
    y = fem.apply_masked(c["K"], c["fixed"], v)
    assert np.array_equal(y[c["fixed"]], v[c["fixed"]])
    v0 = v.copy()
    v0[c["fixed"]] = 0
    assert np.allclose(y[~c["fixed"]], (c["K"] @ v0)[~c["fixed"]], rtol=0, atol=1e-13)


@pytest.mark.parametrize("bc", [grid.BC_CANTILEVER, grid.BC_MBB])
def test_sensitivity_central_differences(bc):
    """Eq. 3 against central differences of c(x) = f^T u(x)."""
    nelx, nely, nelz = 6, 3, 3
    rng = np.random.default_rng(7)
    x = rng.uniform(0.2, 1.0, nelx * nely * nelz)
    E0, Emin, p = 1.0, 1e-9, 3.0
    K0 = element.k0(0.3, 1.0)
    fixed, f = fem.problem_arrays(nelx, nely, nelz, bc)

    def comp(xv):
        K = fem.assemble(nelx, nely, nelz, fem.modulus(xv, E0, Emin, p), K0)
        return fem.compliance(f, fem.solve_direct(K, f, fixed))

    K = fem.assemble(nelx, nely, nelz, fem.modulus(x, E0, Emin, p), K0)
    u = fem.solve_direct(K, f, fixed)
    dc = fem.sensitivity(x, fem.element_energy(nelx, nely, nelz, K0, u), E0, Emin, p)
    assert np.all(dc <= 0)
    for e in rng.choice(x.size, 8, replace=False):
        d = 1e-4 * x[e]
        xp, xm = x.copy(), x.copy()
        xp[e] += d
        xm[e] -= d
        fd = (comp(xp) - comp(xm)) / (2 * d)
        assert abs(fd - dc[e]) <= 1e-6 * abs(dc).max()


def test_mbb_is_nonsingular_with_y_pin():
    nelx, nely, nelz = 4, 2, 2
    K = fem.assemble(nelx, nely, nelz, np.ones(16), element.k0(0.3, 1.0))
    fixed, f = fem.problem_arrays(nelx, nely, nelz, grid.BC_MBB)
    free = np.flatnonzero(~fixed)
    ev = np.linalg.eigvalsh(K[free][:, free].toarray())
    assert ev[0] > 1e-6
    # without the y pin the y translation is a null mode
    fixed2 = fixed.copy()
    fixed2[1] = False
    free2 = np.flatnonzero(~fixed2)
    ev2 = np.linalg.eigvalsh(K[free2][:, free2].toarray())
    assert abs(ev2[0]) < 1e-10


def test_load_shares_sum_to_total():
    for bc in (grid.BC_CANTILEVER, grid.BC_MBB):
        f = grid.load_vector(7, 5, 3, bc, 2.5)
        assert abs(f[2::3].sum() + 2.5) < 1e-15 and not f[0::3].any() and not f[1::3].any()


def test_apply_rows_matches_assembled_operator():
    nelx, nely, nelz = 5, 4, 3
    rng = np.random.default_rng(4)
    E = rng.uniform(0.1, 1.0, nelx * nely * nelz)
    K0 = element.k0(0.3, 1.0)
    K = fem.assemble(nelx, nely, nelz, E, K0)
    for bc in (grid.BC_CANTILEVER, grid.BC_MBB):
        fixed, _ = fem.problem_arrays(nelx, nely, nelz, bc)
        u = rng.standard_normal(fixed.size)
        y = fem.apply_masked(K, fixed, u).reshape(-1, 3)
        nodes = np.arange(y.shape[0])
        yr = fem.apply_rows(nelx, nely, nelz, E, K0, u, fixed, nodes)
        assert np.max(np.abs(y - yr)) < 1e-14
