"""Writes tests/golden/paper_simp_oracle.json: the oracle's SIMP loop on the
paper's two benchmark problems (40 x 20 x 20 voxels, h = 0.05, V_f = 0.4,
p = 3, R = 2 elements, textbook OC) stopped at Delta rho_max = 8 % and 4 %,
with the state solved by the oracle's Jacobi-PCG to 1e-10.  Calls only
oracle/; each case runs in its own process (about ten minutes on one core).

    python tests/golden/make_paper_simp.py
"""
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

CASES = [("cantilever_corners", 3, 0.08), ("cantilever_corners", 3, 0.04),
         ("mbb_strip", 4, 0.08), ("mbb_strip", 4, 0.04)]


def run(case):
    from oracle import simp
    name, bc, tol = case
    x, hist = simp.simp_run(40, 20, 20, vf=0.4, rmin=2.0, h=0.05, bc=bc, change_tol=tol,
                            max_iters=200, method="pcg", rtol=1e-10)
    return name, tol, {"iterations": len(hist), "c": [r["c"] for r in hist],
                       "change": [r["change"] for r in hist],
                       "volume": [r["volume"] for r in hist]}


if __name__ == "__main__":
    out = {"source": "oracle.simp.simp_run, 40x20x20, h = 0.05, vf 0.4, rmin 2, "
                     "state by oracle Jacobi-PCG to 1e-10 (written by tests/golden/make_paper_simp.py)"}
    with ProcessPoolExecutor(max_workers=4) as ex:
        for name, tol, rec in ex.map(run, CASES):
            out.setdefault(name, {})[str(tol)] = rec
            print(name, tol, rec["iterations"], rec["c"][-1], flush=True)
    with open(os.path.join(HERE, "paper_simp_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
