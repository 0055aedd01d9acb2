"""Host-side checks of the C ABI that need no GPU: the built library loads,
exports every function include/to.h declares, and validates problems."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2605_04735_amd import _lib as L
from paper_2605_04735_amd import api as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "to.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(to_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert "to_solve" in names and "to_density_to_sdf" in names
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (to_[a-z0-9_]+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    lib = L.lib()
    for n in names:
        assert getattr(lib, n) is not None


def test_workspace_size_validates_problem():
    assert A.to_workspace_size(A.Problem(24, 12, 6)) > 0
    big = A.to_workspace_size(A.Problem(96, 48, 48))
    assert big > 0.69e6 * 6 * 8
    mixed = A.to_workspace_size(A.Problem(96, 48, 48, precision=A.PREC_FP32_REFINE))
    assert mixed < big
    bad = [dict(nelx=0), dict(h=0.0), dict(nu=0.5), dict(Emin=2.0), dict(penal=0.5),
           dict(bc=7), dict(rtol=0.0), dict(max_iters=0), dict(precision=9)]
    for kw in bad:
        args = dict(nelx=4, nely=3, nelz=2)
        args.update(kw)
        with pytest.raises(A.TopoError) as e:
            A.to_workspace_size(A.Problem(**args))
        assert e.value.status == L.TO_E_INVALID
    with pytest.raises(A.TopoError):
        A.to_workspace_size(A.Problem(4, 3, 2, bc=A.BC_CUSTOM))
    # limits: float64 vectors below 2^31 bytes, the product's x-y tiles within
    # its block bound; both rejected before any device work
    for dims in [(500, 500, 400), (2000, 2000, 1)]:
        with pytest.raises(A.TopoError) as e:
            A.to_workspace_size(A.Problem(*dims))
        assert e.value.status == L.TO_E_INVALID
    # dimensions whose node counts overflow 32-bit ints are rejected, not wrapped
    INT_MAX = 2 ** 31 - 1
    for dims in [(INT_MAX, 1, 1), (1, INT_MAX, 1), (1, 1, INT_MAX), (INT_MAX,) * 3]:
        with pytest.raises(A.TopoError) as e:
            A.to_workspace_size(A.Problem(*dims))
        assert e.value.status == L.TO_E_INVALID
    # the largest accepted grids size normally
    assert A.to_workspace_size(A.Problem(440, 440, 440)) > 0
    assert A.to_workspace_size(A.Problem(1200, 1200, 2)) > 0


STRUCTS = [(L.ToProblem, "to_problem"), (L.ToSolveInfo, "to_solve_info"),
           (L.ToOcInfo, "to_oc_info"), (L.ToSimpParams, "to_simp_params"),
           (L.ToSimpInfo, "to_simp_info")]


def test_struct_layout_matches_header(tmp_path):
    """ctypes field offsets and sizes equal the C compiler's for include/to.h."""
    body, expect = "", []
    for cls, cname in STRUCTS:
        for f, _ in cls._fields_:
            body += 'printf("%%zu ", offsetof(%s, %s));' % (cname, f.rstrip("_"))
            expect.append(getattr(cls, f).offset)
        body += 'printf("%%zu ", sizeof(%s));' % cname
        expect.append(ctypes.sizeof(cls))
    src = tmp_path / "lay.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "to.h"\n'
                   'int main(void){ %s return 0; }' % body)
    exe = tmp_path / "lay"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    assert vals == expect


def test_last_error_without_context():
    with pytest.raises(A.TopoError):
        A.to_workspace_size(A.Problem(-1, 3, 2))
    assert "grid" in A.L.lib().to_last_error(None).decode()


def test_null_context_is_rejected_before_any_device_work():
    """Every call that takes a context returns TO_E_INVALID for NULL, with a
    message, and touches no device (this runs without a GPU)."""
    lib = L.lib()
    P = ctypes.c_void_p
    calls = {
        "to_solve": (None, None, None, None, None),
        "to_compliance_sensitivity": (None, None, None, None, None),
        "to_filter": (None, ctypes.c_double(1.5), 0, None, None, None),
        "to_density_to_sdf": (None, None, ctypes.c_double(0.5), None, None, None),
        "to_oc_update": (None, None, None, ctypes.c_double(0.4), ctypes.c_double(0.2),
                         ctypes.c_double(0.5), None, None),
        "to_simp": (None, None, None, None, None, None, None),
        "to_ls_advect": (None, None, None, ctypes.c_double(0.5), 1, None),
        "to_ls_reinit": (None, None, ctypes.c_double(0.5), ctypes.c_double(1e-3), 10, None, None),
        "to_shape_rhs": (None, None, None, ctypes.c_double(2.0), ctypes.c_double(1.0),
                         ctypes.c_double(0.0), None),
        "to_hilbert_extend": (None, ctypes.c_double(1.0), None, None, ctypes.c_double(1e-8), 10,
                              None, None),
        "to_volume_fraction": (None, None, None),
        "to_matvec": (None, None, None, None),
        "to_matvec_f32": (None, None, None, None),
    }
    for name, args in calls.items():
        st = getattr(lib, name)(*args)
        assert st == L.TO_E_INVALID, name
        assert lib.to_last_error(None), name


STALL_DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include "refine_rule.h"
// reads residuals from argv, prints the index of the first stalled record (-1: none)
int main(int argc, char **argv) {
  topo::StagnationRule r;
  for (int i = 1; i < argc; ++i)
    if (r.record(std::atof(argv[i]))) { std::printf("%d\n", i - 1); return 0; }
  std::printf("-1\n");
  return 0;
}
"""


def test_refinement_stagnation_rule(tmp_path):
    """The refinement's attainable-accuracy stop, compiled on its own from the
    header both the one-design solve and the server use: it fires only when the
    residual after pass n is not below half the residual after pass n - 4."""
    src = tmp_path / "stall.cpp"
    src.write_text(STALL_DRIVER)
    exe = tmp_path / "stall"
    subprocess.run(["g++", "-std=c++17", "-I", os.path.join(ROOT, "paper_2605_04735_amd", "csrc"),
                    str(src), "-o", str(exe)], check=True)

    def first_stall(seq):
        out = subprocess.run([str(exe)] + ["%.17g" % v for v in seq], capture_output=True,
                             text=True, check=True).stdout
        return int(out)

    # slow but steady progress: 0.84 per pass halves the residual in four passes
    # (0.84^4 = 0.498), so it never stalls; a three-pass window (0.84^3 = 0.593)
    # would have stopped it at the fourth pass
    assert first_stall([0.84 ** k for k in range(40)]) == -1
    # progress that stops: flat after the third pass
    seq = [1.0, 0.1, 0.01, 0.005, 0.005, 0.005, 0.005, 0.005, 0.005]
    # records 3..6 compare with 1.0, 0.1, 0.01, 0.005 (four back): the first
    # that is not below half of it is record 7 (0.005 vs 0.005 / 2 at record 3)
    assert first_stall(seq) == 7
    # exactly half four passes back does not stall; just above half does
    assert first_stall([1.0, 0.9, 0.8, 0.7, 0.5]) == -1
    assert first_stall([1.0, 0.9, 0.8, 0.7, 0.5000001]) == 4
    # a NaN residual counts as no progress
    assert first_stall([1.0, 0.9, 0.8, 0.7, float("nan")]) == 4
    # fewer than five records never stall
    assert first_stall([1.0, 1.0, 1.0, 1.0]) == -1


PREDICT_DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include "stop_predict.h"
int main(int argc, char **argv) {
  // q0 s0 q1 s1 target
  const double v = topo::predicted_steps(std::atof(argv[1]), std::atof(argv[2]), std::atof(argv[3]),
                                         std::atof(argv[4]), std::atof(argv[5]));
  std::printf("%.17g\n", v);
  return 0;
}
"""


def test_stop_prediction(tmp_path):
    """The host's guess of the remaining steps of a device loop (the inner CG,
    the extension CG and reinitialisation queue about that many launches),
    compiled on its own from the header the library uses: exact for a
    geometric sequence, and no guess (+inf) where nothing decays."""
    src = tmp_path / "predict.cpp"
    src.write_text(PREDICT_DRIVER)
    exe = tmp_path / "predict"
    subprocess.run(["g++", "-std=c++17", "-I", os.path.join(ROOT, "paper_2605_04735_amd", "csrc"),
                    str(src), "-o", str(exe)], check=True)

    def steps(q0, s0, q1, s1, target):
        out = subprocess.run([str(exe)] + ["%.17g" % v for v in (q0, s0, q1, s1, target)],
                             capture_output=True, text=True, check=True).stdout
        return float(out)

    # q = 2^-s seen at steps 10 and 20: 2^-30 is 10 steps away, 2^-25 five
    assert abs(steps(2.0 ** -10, 10, 2.0 ** -20, 20, 2.0 ** -30) - 10.0) < 1e-9
    assert abs(steps(2.0 ** -10, 10, 2.0 ** -20, 20, 2.0 ** -25) - 5.0) < 1e-9
    # slower decay, 0.9 per step from step 0: 0.9^100 from 0.9^32 is 68 steps
    assert abs(steps(1.0, 0, 0.9 ** 32, 32, 0.9 ** 100) - 68.0) < 1e-9
    # already at or below the target: no steps left
    assert steps(1.0, 0, 1e-3, 10, 1e-2) < 0.0
    assert steps(1.0, 0, 1e-3, 10, 1e-3) == 0.0
    inf = float("inf")
    # nothing to extrapolate: no decay, no step between the looks, bad values
    assert steps(1.0, 0, 1.0, 10, 1e-3) == inf
    assert steps(1.0, 0, 2.0, 10, 1e-3) == inf
    assert steps(1.0, 10, 0.5, 10, 1e-3) == inf
    assert steps(0.0, 0, 0.5, 10, 1e-3) == inf
    assert steps(inf, 0, 0.5, 10, 1e-3) == inf
    assert steps(1.0, 0, 0.5, 10, 0.0) == inf
    assert steps(float("nan"), 0, 0.5, 10, 1e-3) == inf
