"""SIMP design loop with the optimality-criteria (OC) update (oracle, test
infrastructure only).

The paper's first stage (Sec. 2.1, with the set-up of Sec. 4) runs SIMP from a
uniform density equal to the target volume fraction V_f, with penalisation
p = 3, the sensitivity filter of Eq. 4 at radius R = 2h, and the OC update of
the densities; it stops when the largest density change of an iteration,
Delta rho_max, falls below a threshold (0.5 % to 8 % in its tests).

The paper names OC (Bendsoe and Sigmund's textbook scheme) but not its
parameters, so the textbook values are taken:

  * heuristic fixed-point update with damping eta = 1/2 and move limit 0.2:
        B_e    = -dc_e / lambda                      (unit volume derivative)
        x_new  = clamp(x_e B_e^eta, [max(0, x_e - move), min(1, x_e + move)])
    A positive sensitivity (never produced by compliance) is taken as zero,
    so such an element can only lose material.
  * lambda by bisection on [0, 1e9]: the midpoint is evaluated, and the
    bracket's lower end moves up when the new design holds more material than
    V_f times the element count, else its upper end moves down; the loop ends
    once (l2 - l1) / (l1 + l2) <= 1e-3.  The design returned is the one of the
    last midpoint evaluated.  When the target cannot be met from above (every
    sensitivity zero, say) the lower end never leaves 0 and the loop would only
    end by underflow; more than 200 midpoints is an error.
  * the lower density bound is 0 (E_min > 0 keeps K regular), as in the
    modified SIMP of Eq. 1.

  oc_update   one OC update with its bisection
  simp_run    solve -> compliance and sensitivity -> sensitivity filter -> OC,
              until Delta rho_max <= tol or an iteration cap
"""
import numpy as np

from . import fem, filters

OC_MOVE = 0.2
OC_ETA = 0.5
OC_L2 = 1e9
OC_TOL = 1e-3
OC_MAX_STEPS = 200


def oc_candidate(x, dc, lam, move=OC_MOVE, eta=OC_ETA):
    """The OC design for one multiplier value lam."""
    x = np.asarray(x, dtype=np.float64)
    b = np.maximum(-np.asarray(dc, dtype=np.float64), 0.0) / lam
    t = x * (np.sqrt(b) if eta == 0.5 else b ** eta)
    lo = np.maximum(0.0, x - move)
    hi = np.minimum(1.0, x + move)
    return np.maximum(lo, np.minimum(hi, t))


def oc_update(x, dc, vf, move=OC_MOVE, eta=OC_ETA, l2=OC_L2, tol=OC_TOL, max_steps=OC_MAX_STEPS):
    """One OC update.  Returns (x_new, lam, steps): the design of the last
    midpoint evaluated, that midpoint, and the number of midpoints.  Raises
    RuntimeError after max_steps midpoints."""
    x = np.asarray(x, dtype=np.float64)
    dc = np.asarray(dc, dtype=np.float64)
    if not (np.all(np.isfinite(x)) and np.all(np.isfinite(dc))):
        raise ValueError("non-finite x or dc")
    if np.any(x < 0.0) or np.any(x > 1.0):
        raise ValueError("x outside [0, 1]")
    target = vf * x.size
    l1 = 0.0
    steps = 0
    xnew, lam = None, None
    while (l2 - l1) / (l1 + l2) > tol:
        if steps == max_steps:
            raise RuntimeError("OC bisection: no multiplier after %d midpoints" % steps)
        lam = 0.5 * (l2 + l1)
        xnew = oc_candidate(x, dc, lam, move, eta)
        steps += 1
        if xnew.sum() > target:
            l1 = lam
        else:
            l2 = lam
    return xnew, lam, steps


def simp_run(nelx, nely, nelz, *, vf=0.4, rmin=2.0, penal=3.0, E0=1.0, Emin=1e-9, nu=0.3,
             h=1.0, bc=0, load_total=1.0, move=OC_MOVE, eta=OC_ETA, change_tol=0.01,
             max_iters=50, x0=None, method="direct", rtol=1e-12):
    """The SIMP loop.  Returns (x, history) where history holds, per design
    iteration, the compliance of the design solved, the largest density
    change of the update that followed, the volume fraction after it, and the
    OC multiplier.  method: the state solve, "direct" or "pcg" (to rtol)."""
    nel = nelx * nely * nelz
    x = np.full(nel, float(vf)) if x0 is None else np.array(x0, dtype=np.float64)
    hist = []
    for _ in range(max_iters):
        _, c, dc, _ = fem.full_solve(nelx, nely, nelz, x, h=h, E0=E0, Emin=Emin, nu=nu,
                                     penal=penal, bc=bc, load_total=load_total, method=method,
                                     rtol=rtol)
        dcf = filters.sensitivity_filter(x, dc, nelx, nely, nelz, rmin, h)
        xnew, lam, steps = oc_update(x, dcf, vf, move, eta)
        change = float(np.max(np.abs(xnew - x)))
        x = xnew
        hist.append({"c": c, "change": change, "volume": float(x.mean()), "lam": lam,
                     "steps": steps})
        if change <= change_tol:
            break
    return x, hist
