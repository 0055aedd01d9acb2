"""Pins for the oracle's OC update and SIMP loop (Sec. 2.1, the SIMP set-up of
Sec. 4; OC in its textbook form).

  * exact bisection: on a uniform design the multiplier sequence follows from
    integer arithmetic alone, which fixes every midpoint and the step count;
  * closed form: when no bound is active the OC design is x (B/lam)^eta and the
    volume condition gives lam = (sum x (-dc)^eta / (V_f n))^(1/eta); the
    bisection must land within its own bracket of it;
  * the move limit and the [0, 1] box, a uniform fixed point, the step cap on
    an unreachable target;
  * on the cantilever, whose loads and supports are mirror-symmetric in y, the
    SIMP designs stay mirror-symmetric, the volume stays at V_f, no density
    moves more than the move limit and the compliance drops."""
import numpy as np
import pytest

from oracle import simp, fem, filters


def _near_uniform(n, seed, eta):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.38, 0.42, n)
    dc = -1e-2 * (1.0 + 0.02 * rng.uniform(-1.0, 1.0, n))
    lam_star = (np.sum(x * (-dc) ** eta) / (0.4 * n)) ** (1.0 / eta)
    return x, dc, lam_star


@pytest.mark.parametrize("eta", [0.5, 0.3])
def test_closed_form_multiplier(eta):
    x, dc, lam_star = _near_uniform(1000, 3, eta)
    xnew, lam, steps = simp.oc_update(x, dc, 0.4, eta=eta)
    # the bracket holding both lam and lam_star is at most 1e-3 (l1 + l2) wide
    assert abs(lam - lam_star) <= 2.001e-3 * lam_star
    t = x * (-dc / lam) ** eta
    assert np.all(t > x - 0.2) and np.all(t < x + 0.2)      # no bound active
    assert np.max(np.abs(xnew - t)) <= 1e-15
    assert abs(xnew.sum() / (0.4 * x.size) - 1.0) <= eta * 2.5e-3
    # the bisection from [0, 1e9] needs log2(1e9 / lam) steps to reach the
    # root's octave and about 10 more to reach a 1e-3 bracket
    assert abs(steps - (np.log2(1e9 / lam_star) + 10)) <= 2


@pytest.mark.parametrize("d", [0.0123456789, 3.75e-7, 42.0001])
def test_midpoints_are_exact_bisection(d):
    # uniform x = V_f and dc = -d: the design holds more than V_f exactly when
    # lam < d, so after k halvings of [0, 1e9] the bracket is
    # [a, a + 1] 1e9 / 2^k with a = floor(d 2^k / 1e9), the loop stops at the
    # first k with 1 / (2 a + 1) <= 1e-3, and the last midpoint evaluated is
    # (2 a_(k-1) + 1) 1e9 / 2^k -- all in exact rational arithmetic
    from fractions import Fraction
    n = 64
    _, lam, steps = simp.oc_update(np.full(n, 0.4), np.full(n, -d), 0.4)
    def a(k):
        return (Fraction(d) * 2 ** k) // 10 ** 9
    k = 1
    while 2 * a(k) + 1 < 1000:
        k += 1
    assert steps == k
    assert lam == float(Fraction((2 * a(k - 1) + 1) * 10 ** 9, 2 ** k))


def test_returns_the_last_midpoint_design():
    rng = np.random.default_rng(5)
    x = rng.uniform(0.0, 1.0, 300)
    dc = -10.0 ** rng.uniform(-4, 0, 300)
    xnew, lam, _ = simp.oc_update(x, dc, 0.5)
    assert np.array_equal(xnew, simp.oc_candidate(x, dc, lam))


def test_move_and_box_limits():
    rng = np.random.default_rng(7)
    x = rng.uniform(0.0, 1.0, 2000)
    dc = -10.0 ** rng.uniform(-6, 0, 2000)
    x[:10], dc[:10] = 0.1, 0.0        # no sensitivity: down to the box bound 0
    xnew, _, _ = simp.oc_update(x, dc, 0.45)
    lo, hi = np.maximum(0.0, x - 0.2), np.minimum(1.0, x + 0.2)
    assert np.all(xnew >= lo) and np.all(xnew <= hi)
    assert np.sum(xnew == lo) > 50 and np.sum(xnew == hi) > 50
    assert np.all(xnew[:10] == 0.0) and np.sum(xnew == 1.0) > 0
    # a larger sensitivity never gets less material from the same x
    xs = np.full(50, 0.5)
    d = -np.linspace(1e-3, 1e-1, 50)
    xn, _, _ = simp.oc_update(xs, d, 0.5)
    assert np.all(np.diff(xn) >= 0.0) and xn[-1] > xn[0]


def test_positive_sensitivity_only_loses_material():
    x = np.full(10, 0.5)
    dc = -np.ones(10)
    dc[3] = 2.0
    xnew, _, _ = simp.oc_update(x, dc, 0.5)
    assert xnew[3] == 0.3


def test_uniform_fixed_point():
    x = np.full(512, 0.4)
    xnew, lam, _ = simp.oc_update(x, np.full(512, -0.05), 0.4)
    assert np.all(xnew == xnew[0]) and abs(xnew[0] / 0.4 - 1.0) <= 1.5e-3
    assert abs(lam / 0.05 - 1.0) <= 2.001e-3


def test_unreachable_target_is_an_error():
    with pytest.raises(RuntimeError):
        simp.oc_update(np.full(20, 0.5), np.zeros(20), 0.5)
    with pytest.raises(ValueError):
        simp.oc_update(np.array([0.5, np.nan]), np.array([-1.0, -1.0]), 0.5)
    with pytest.raises(ValueError):
        simp.oc_update(np.array([0.5, 1.5]), np.array([-1.0, -1.0]), 0.5)


def test_simp_cantilever_invariants():
    nelx, nely, nelz = 12, 6, 4
    x, hist = simp.simp_run(nelx, nely, nelz, vf=0.4, rmin=2.0, change_tol=0.01, max_iters=60)
    assert 10 < len(hist) < 60 and hist[-1]["change"] <= 0.01
    for hrec in hist:
        assert abs(hrec["volume"] / 0.4 - 1.0) <= 1.5e-3
        assert hrec["change"] <= 0.2 + 1e-15
    assert hist[-1]["c"] < 0.4 * hist[0]["c"]
    # loads and supports are mirror-symmetric in y, and so are K0 and the
    # filter stencil: the design must be too
    g = x.reshape(nelz, nely, nelx)
    assert np.max(np.abs(g - g[:, ::-1, :])) < 1e-9
    assert np.max(g) == 1.0 and np.min(g) < 0.1


def test_simp_first_iteration_and_stop_rule():
    nelx, nely, nelz = 8, 4, 3
    x, hist = simp.simp_run(nelx, nely, nelz, vf=0.4, rmin=2.0, change_tol=0.25, max_iters=5)
    assert len(hist) == 1 and hist[0]["change"] <= 0.2 + 1e-15
    x0 = np.full(nelx * nely * nelz, 0.4)
    _, c, dc, _ = fem.full_solve(nelx, nely, nelz, x0)
    x1, _, _ = simp.oc_update(x0, filters.sensitivity_filter(x0, dc, nelx, nely, nelz, 2.0), 0.4)
    assert np.array_equal(x, x1) and c == hist[0]["c"]
