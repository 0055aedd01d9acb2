#!/usr/bin/env python3
"""Benchmark of the voxel hex8 topology-optimisation hot path on one MI355X.

Workload (the configuration the metric is quoted on): a 96 x 48 x 48 hex8
cantilever (698,691 DOF), densities from a seeded Gaussian random field
(length scale 6 elements, sigmoid slope 2, seed 1) in [1e-3, 1], E0 = 1,
Emin = 1e-9, nu = 0.3, p = 3, x = 0 face clamped, unit downward line load on
the bottom edge of the x = 96 face.

One step = one pass of the whole hot path on that design, inputs resident in
HBM: state solve from a zero start (float32 inner Jacobi-PCG + float64 outer
refinement), compliance and sensitivity, density filter (rmin 1.5) and
sensitivity filter (R = 2), density -> SDF with the ersatz volume fraction.
The plain float64 solve is timed the same way.  Both paths stop at the
loosest outer residual that brings compliance, sensitivities and the
displacement (in the energy norm of Eq. 2) within 0.5e-6 of a tight float64
reference on calibration seeds (11, 12, 13), tightened by a further factor of
10 (the error/residual ratio varies between designs), chosen before timing;
the achieved errors of the timed design against the oracle's solution are
reported.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "K*u GDOF/s + solves/s, p50/p99 latency: FP32+refine vs FP64 at rel err 1e-6"
DIMS = (96, 48, 48)
LARGE = (256, 128, 128)
RTOL_LADDER = [1e-3, 3e-4, 1e-4, 3e-5, 1e-5, 3e-6, 1e-6, 3e-7, 1e-7, 3e-8, 1e-8]
TARGET = 1e-6
CAL_MARGIN = 0.5          # calibrate to half the target: residuals are a loose proxy
CAL_SAFETY = 1e-1         # and use a tolerance one decade below the calibrated rung,
RTOL_FLOOR = 1e-8         # but not below 1e-8: float64 itself cannot resolve residuals much
                          # below ~1e-9 of designs whose stiff parts float in near-void
HBM_PEAK_GBS = 8000.0


def cg_bytes_f32(zfuse):
    """Algorithmic bytes per node of the float32 inner-CG kernels: the product
    (which also reads 4 per element, E) and the update by how it treats x.
    With z formed in the product (zfuse) the product reads r, the Jacobi
    diagonal and p_old (28) and writes p and q (24); with z stored it reads z
    and p_old (24) and writes p and q, and every update also writes z (12).
    The update reads r, q, the diagonal and the mask byte (29) and writes r
    (12); advancing x every iteration adds x and p (24) read and x written
    (12); with x grouped, three of four (one of two) updates skip x and the
    fourth (second) reads x and all the group's directions and writes x."""
    zs = 0 if zfuse else 12
    return {"product": 52 if zfuse else 48, "each": 77 + zs, "skip": 41 + zs,
            "flush2": 89 + zs, "flush4": 113 + zs}


def cg_iteration_bytes_f32(zfuse):
    """Per node and iteration, float32 CG as the solve runs it (x grouped by
    two): the product plus the mean of a skipping and a grouped update."""
    b = cg_bytes_f32(zfuse)
    return b["product"] + (b["skip"] + b["flush2"]) / 2


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the 256x128x128 product timing")
    ap.add_argument("--cpu-iters", type=int, default=300)
    ap.add_argument("--no-serving", action="store_true", help="skip the request-stream benchmark")
    ap.add_argument("--no-simp", action="store_true", help="skip the SIMP-loop workload")
    ap.add_argument("--no-levelset", action="store_true",
                    help="skip the level-set evolution/reinitialisation workload")
    ap.add_argument("--no-shape", action="store_true",
                    help="skip the shape-derivative / Hilbertian-extension workload")
    ap.add_argument("--no-paper", action="store_true",
                    help="skip the SIMP stage on the paper's own two problems")
    ap.add_argument("--requests", type=int, default=128)
    ap.add_argument("--no-config0", action="store_true", help="skip the 24x12x6 latency line")
    ap.add_argument("--probe", choices=["copy", "cg", "cg3", "product", "levelset", "shape"],
                    default=None,
                    help="short runs for hardware-counter passes: a device copy of known size, "
                         "one workload solve, products on 256x128x128, or level-set steps on "
                         "its node grid")
    ap.add_argument("--profile-commands", metavar="DIR", default=None,
                    help="print the rocprofv3 commands whose CSV output (under DIR) "
                         "--summarize reduces, one per line, and exit")
    ap.add_argument("--summarize", metavar="DIR", default=None,
                    help="reduce the rocprofv3 CSV output under DIR to the summaries in "
                         "profiles/ and exit (no GPU needed)")
    return ap.parse_args()


COPY_BYTES = 1 << 30


def probe(kind):
    """Short, fixed workloads for rocprofv3 counter passes (no timing)."""
    import torch
    from paper_2605_04735_amd import api as A
    from paper_2605_04735_amd import inputs
    dev = torch.device("cuda:0")
    if kind == "copy":
        a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copy probe: 5 copies of %d bytes (read %d, write %d each)" % (COPY_BYTES, COPY_BYTES,
                                                                             COPY_BYTES))
        return
    if kind in ("cg", "cg3"):
        dims, seed, rtol = (DIMS, 1, 1e-4) if kind == "cg" else (LARGE, 3, 1e-2)
        x = torch.from_numpy(inputs.random_field(*dims, seed=seed, ell=6.0, kappa=2.0)).to(dev)
        ctx = A.to_create(A.Problem(*dims, precision=A.PREC_FP32_REFINE, rtol=rtol))
        u, info, _ = A.to_solve(ctx, x)
        torch.cuda.synchronize()
        log("cg probe: %s" % info)
        return
    if kind == "shape":
        ctx = A.to_create(A.Problem(*LARGE))
        nn = (LARGE[0] + 1) * (LARGE[1] + 1) * (LARGE[2] + 1)
        phi = torch.from_numpy(inputs.sphere_union(*LARGE, 5, scale=2.5)).to(dev)
        u = torch.from_numpy(1e-2 * inputs.random_vector(3 * nn, 5)).to(dev)
        g = A.to_shape_rhs(ctx, phi, u=u, eta=2.0)
        A.to_hilbert_extend(ctx, g, ell=2.0, rtol=1e-8)
        torch.cuda.synchronize()
        log("shape probe done")
        return
    if kind == "levelset":
        ctx = A.to_create(A.Problem(*LARGE))
        phi = torch.from_numpy(inputs.sphere_union(*LARGE, 5, scale=2.5)).to(dev)
        v = torch.from_numpy(inputs.smooth_speed(*LARGE, 7)).to(dev)
        A.to_ls_advect(ctx, phi, v, gamma=0.5, nsteps=10)
        A.to_ls_reinit(ctx, phi, gamma=0.5, tol=1e-3, max_steps=40, raise_on_error=False)
        torch.cuda.synchronize()
        log("level-set probe done")
        return
    # float32 (vector-ALU modal form), float32 on the matrix cores (opt-in
    # variant, TOPO_MFMA=1), float64
    for f32, mfma in ((True, False), (True, True), (False, False)):
        if mfma:
            os.environ["TOPO_MFMA"] = "1"
        p = A.Problem(*LARGE, precision=A.PREC_FP32_REFINE if f32 else A.PREC_FP64)
        ctx = A.to_create(p)
        os.environ.pop("TOPO_MFMA", None)
        u = torch.randn(p.ndof, dtype=torch.float32 if f32 else torch.float64, device=dev)
        y = torch.empty_like(u)
        x = torch.from_numpy(inputs.random_field(*LARGE, seed=3, ell=6.0)).to(dev)
        mv = A.to_matvec_f32 if f32 else A.to_matvec
        mv(ctx, x, u, y)
        for _ in range(10):
            mv(ctx, None, u, y)
        torch.cuda.synchronize()
        ctx.close()
    log("product probe done")


def measured_traffic(summary, kernel, profiles_dir=None):
    """HBM bytes per launch of `kernel` from a committed counter summary, or
    None when the product's sources changed since the counters were taken."""
    try:
        text = open(os.path.join(profiles_dir or PROFILES_DIR, summary)).read()
    except OSError:
        return None
    sha = _source_sha(PRODUCT_SOURCES)
    for sec in text.split("## ")[1:]:
        fields = dict(l.split(": ", 1) for l in sec.splitlines() if ": " in l)
        if fields.get("kernel", "").strip() != kernel or "traffic_bytes_per_launch" not in fields:
            continue
        if sha not in fields.get("source", ""):
            return None
        return float(fields["traffic_bytes_per_launch"])
    return None


def profiled_avg_us(summary, kernel, profiles_dir=None):
    """rocprofv3 average duration (us) of `kernel` from the kernel table of a
    committed trace summary, or None when the product's sources changed since
    the trace was taken."""
    try:
        lines = open(os.path.join(profiles_dir or PROFILES_DIR, summary)).read().splitlines()
    except OSError:
        return None
    sha = _source_sha(PRODUCT_SOURCES)
    if not any(l.startswith("source:") and sha in l for l in lines[:3]):
        return None
    cols = None  # the column names while inside the kernel table (it ends at a blank line)
    for l in lines:
        if l.startswith("kernel ") and "avg_us" in l:
            cols = l.split()[1:]
            continue
        if not l.strip():
            cols = None
        if cols is None:
            continue
        parts = l.rsplit(None, len(cols))
        if len(parts) == len(cols) + 1 and (parts[0] == kernel or parts[0].startswith(kernel + "(")):
            return float(dict(zip(cols, parts[1:]))["avg_us"])
    return None


def rel2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ---------------------------------------------------------------- profiles
# The rocprofv3 runs behind profiles/, and their reduction.  Every run is one
# committed command (a probe of this file, or the bench step itself); the
# summaries are regenerated with --summarize from the CSV files the runs wrote.
SQ_COUNTERS = ("SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS SQ_INSTS_SALU SQ_LDS_BANK_CONFLICT "
               "SQ_ACTIVE_INST_VALU SQ_BUSY_CYCLES SQ_WAVE_CYCLES")
SQ_MFMA_COUNTERS = "SQ_INSTS_VALU_MFMA_MOPS_BF16 SQ_VALU_MFMA_BUSY_CYCLES SQ_INSTS_MFMA SQ_BUSY_CU_CYCLES"
# the bench's large workloads only (products at 256x128x128, the config-2 MBB,
# the 256x128x128 solves): the command whose live CG-product timing is the
# top-level roofline
BENCH_LARGE_ARGS = ("--steps 1 --warmup 1 --no-cpu-baseline --no-serving --no-simp --no-levelset "
                    "--no-shape --no-paper --no-config0")
BENCH_TRACE_ARGS = ("--steps 5 --warmup 1 --no-cpu-baseline --no-serving --no-large --no-simp "
                    "--no-levelset --no-shape --no-paper --no-config0")
PROFILE_RUNS = {  # -o name: (rocprofv3 options, bench.py arguments)
    "copy_fetch": ("--pmc FETCH_SIZE", "--probe copy"),
    "copy_write": ("--pmc WRITE_SIZE", "--probe copy"),
    "product_trace": ("--kernel-trace --stats", "--probe product"),
    "product_fetch": ("--pmc FETCH_SIZE", "--probe product"),
    "product_write": ("--pmc WRITE_SIZE", "--probe product"),
    "product_sq": ("--pmc " + SQ_COUNTERS, "--probe product"),
    "product_mfma": ("--pmc " + SQ_MFMA_COUNTERS, "--probe product"),
    "cg_fetch": ("--pmc FETCH_SIZE", "--probe cg"),
    "cg_write": ("--pmc WRITE_SIZE", "--probe cg"),
    "cg3_trace": ("--kernel-trace --stats", "--probe cg3"),
    "cg3_fetch": ("--pmc FETCH_SIZE", "--probe cg3"),
    "cg3_write": ("--pmc WRITE_SIZE", "--probe cg3"),
    "cg3_sq": ("--pmc " + SQ_COUNTERS, "--probe cg3"),
    "bench_trace": ("--kernel-trace --stats", BENCH_TRACE_ARGS),
    "bench_large_trace": ("--kernel-trace --stats", BENCH_LARGE_ARGS),
    "ls_trace": ("--kernel-trace --stats", "--probe levelset"),
    "ls_fetch": ("--pmc FETCH_SIZE", "--probe levelset"),
    "ls_write": ("--pmc WRITE_SIZE", "--probe levelset"),
    "ls_sq": ("--pmc " + SQ_COUNTERS, "--probe levelset"),
    "shape_trace": ("--kernel-trace --stats", "--probe shape"),
    "shape_fetch": ("--pmc FETCH_SIZE", "--probe shape"),
    "shape_write": ("--pmc WRITE_SIZE", "--probe shape"),
    "shape_sq": ("--pmc " + SQ_COUNTERS, "--probe shape"),
}
# the trace of the bench's large workloads: its average for the inner-CG
# product is reported beside the live roofline figure
LARGE_TRACE = "kernel_trace_bench_large_256x128x128.txt"
PROFILES_DIR = os.path.join(ROOT, "profiles")
PRODUCT_SOURCES = ("k_matvec.hip", "k_mfma.hip", "device_common.h", "common.h")
LS_SOURCES = ("k_levelset.hip", "device_common.h", "common.h")
SHAPE_SOURCES = ("k_shape.hip", "device_common.h", "common.h")


def _nodes(d):
    return (d[0] + 1) * (d[1] + 1) * (d[2] + 1), d[0] * d[1] * d[2]


def cg_zfuse_dims(dims):
    """Whether the library forms the CG z inside the product on grid `dims`."""
    from paper_2605_04735_amd.api import cg_zfuse
    return cg_zfuse(dims)


def algorithmic_bytes(kernel, dims):
    """Bytes one launch of `kernel` must move on grid `dims` (nel voxels, nn
    nodes): every input read once, every output written once."""
    nn, nel = _nodes(dims)
    table = [  # (name fragment, bytes per node, bytes per element)
        ("k_matvec<float, 0>", 25, 4),         # read u (12) and the mask byte, E; write y (12)
        ("k_matvec_mfma<0>", 25, 4),
        ("k_matvec<double, 0>", 49, 8),
        ("k_cg_matvec1<float, false, false, 1>", cg_bytes_f32(True)["product"], 4),
        ("k_cg_matvec1<float, false, true, 1>", cg_bytes_f32(True)["product"], 4),
        ("k_cg_matvec1<float, false, false, 0>", cg_bytes_f32(False)["product"], 4),
        ("k_cg_matvec1<float, false, true, 0>", cg_bytes_f32(False)["product"], 4),
        ("k_cg_update1<float, false, 0>", cg_bytes_f32(cg_zfuse_dims(dims))["each"], 0),
        ("k_cg_update1<float, false, 1>", cg_bytes_f32(cg_zfuse_dims(dims))["skip"], 0),
        ("k_cg_update1<float, false, 2>", cg_bytes_f32(cg_zfuse_dims(dims))["flush2"], 0),
        ("k_cg_update1<float, false, 3>", cg_bytes_f32(cg_zfuse_dims(dims))["flush4"], 0),
        ("k_ls_advect", 24, 0), ("k_ls_reinit", 16, 0),
        ("k_hcg_apply", 17, 0), ("k_hcg_update", 56, 0), ("k_hcg_dir", 24, 0),
        ("__amd_rocclr_copyBuffer", None, None),
    ]
    for frag, bn, be in table:
        if frag in kernel and bn is not None:
            return bn * nn + be * nel
    return None


def profile_commands(outdir):
    return ["rocprofv3 %s --output-format csv -d %s -o %s -- python3 bench.py %s"
            % (opts, outdir, name, args) for name, (opts, args) in PROFILE_RUNS.items()]


def _csv_rows(root, name, suffix):
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(root, "**", "%s*%s" % (name, suffix)), recursive=True)):
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def _durations(root, name):
    """{kernel name: [duration us, ...]} from a kernel-trace run."""
    out = {}
    for r in _csv_rows(root, name, "kernel_trace.csv"):
        k = r.get("Kernel_Name", "")
        out.setdefault(k, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    return out


def _counter(root, name, counter):
    """{kernel name: [value per dispatch, ...]} of one counter."""
    out = {}
    for r in _csv_rows(root, name, "counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        out.setdefault(r.get("Kernel_Name", ""), []).append(float(r["Counter_Value"]))
    return out


def _working(vals):
    """Median over the upper half: launches after a solve's stop return at
    once, so the lower half of a CG kernel's launches measures no work."""
    v = sorted(vals)
    return float(np.median(v[len(v) // 2:])) if v else float("nan")


def _source_sha(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        path = os.path.join(ROOT, "paper_2605_04735_amd", "csrc", f)
        if os.path.exists(path):
            h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def _source_line(files):
    return "source: sha256[:16] of paper_2605_04735_amd/csrc/{%s} = %s" % (",".join(files),
                                                                           _source_sha(files))


def _cmd_lines(names, outdir):
    return ["  rocprofv3 %s --output-format csv -d %s -o %s -- python3 bench.py %s"
            % (PROFILE_RUNS[n][0], outdir, n, PROFILE_RUNS[n][1]) for n in names]


def _copy_scales(root):
    """FETCH_SIZE and WRITE_SIZE scale factors from the copy probe: a copy of
    COPY_BYTES reads and writes COPY_BYTES; each counter is scaled to that."""
    f = _counter(root, "copy_fetch", "FETCH_SIZE")
    w = _counter(root, "copy_write", "WRITE_SIZE")
    kf = [k for k in f if "copyBuffer" in k]
    kw = [k for k in w if "copyBuffer" in k]
    if not kf or not kw:
        return None
    fk, wk = _working(f[kf[0]]), _working(w[kw[0]])
    exp = COPY_BYTES / 1024.0
    return {"fetch_scale": exp / fk, "write_scale": exp / wk, "fetch_kib": fk, "write_kib": wk,
            "kernel": kf[0], "dispatches": (len(f[kf[0]]), len(w[kw[0]]))}


def _committed_scales(profiles_dir=None):
    try:
        text = open(os.path.join(profiles_dir or PROFILES_DIR, "pmc_copy_calibration.txt")).read()
    except OSError:
        return None
    out = {}
    for line in text.splitlines():
        for key in ("fetch_scale", "write_scale"):
            if line.startswith(key + ":"):
                out[key] = float(line.split(":")[1])
    return out if len(out) == 2 else None


# (file, title, dims, trace run, fetch run, write run, sq runs, sources, kernels of interest)
SUMMARIES = [
    ("pmc_product_256x128x128.txt",
     "products y = K u (plain form, fixed DOFs as identity rows) at 256x128x128, random-field "
     "moduli (seed 3); 1 + 10 launches per kernel", LARGE, "product_trace", "product_fetch",
     "product_write", ("product_sq", "product_mfma"), PRODUCT_SOURCES,
     ("k_matvec<float, 0>", "k_matvec_mfma<0>", "k_matvec<double, 0>")),
    ("kernel_trace_cg_256x128x128.txt",
     "one fp32+refine solve of the 256x128x128 cantilever (random-field densities, seed 3) to "
     "rtol 1e-2: inner-CG product and update", LARGE, "cg3_trace", "cg3_fetch", "cg3_write",
     ("cg3_sq",), PRODUCT_SOURCES,
     ("k_cg_matvec1<float, false, false, 1>", "k_cg_matvec1<float, false, true, 1>",
      "k_cg_update1<float, false, 1>", "k_cg_update1<float, false, 2>")),
    (LARGE_TRACE,
     "the bench's large workloads (products at 256x128x128, the config-2 MBB, the 256x128x128 "
     "solves in three precisions), one step of the headline: the inner-CG kernels of the "
     "fp32+refine 256x128x128 solve, the kernel behind the top-level roofline", LARGE,
     "bench_large_trace", None, None, (), PRODUCT_SOURCES,
     ("k_cg_matvec1<float, false, false, 1>", "k_cg_update1<float, false, 1>",
      "k_cg_update1<float, false, 2>")),
    ("pmc_cg_matvec_f32_cantilever_96x48x48.txt",
     "one fp32+refine solve of the 96x48x48 cantilever (seed 1) to rtol 1e-4: inner-CG product "
     "and update (working set resident in the 256 MB Infinity Cache)", DIMS, None, "cg_fetch",
     "cg_write", (), PRODUCT_SOURCES,
     ("k_cg_matvec1<float, false, false, 0>", "k_cg_matvec1<float, false, true, 0>",
      "k_cg_update1<float, false, 1>", "k_cg_update1<float, false, 2>")),
    ("levelset_256x128x128.txt",
     "level-set evolution (10 steps) and reinitialisation (to 1e-3, at most 40 pseudo-steps) on "
     "the 257x129x129 node grid; phi = 2.5 x the distance to three balls, smooth speed of both "
     "signs, CFL number 1/2", LARGE, "ls_trace", "ls_fetch", "ls_write", ("ls_sq",), LS_SOURCES,
     ("k_ls_advect", "k_ls_reinit")),
    ("shape_extension_256x128x128.txt",
     "shape-derivative vector and Hilbertian extension (ell = 2, extension CG to rtol 1e-8) on "
     "the 257x129x129 node grid; phi = 2.5 x the distance to three balls, seeded u", LARGE,
     "shape_trace", "shape_fetch", "shape_write", ("shape_sq",), SHAPE_SOURCES,
     ("k_hcg_apply", "k_hcg_update", "k_hcg_dir", "k_shape_elem", "k_shape_gather")),
]


def summarize(root, out_dir=None):
    """Writes the profiles/ summaries (into `out_dir`, profiles/ by default)
    from the CSV output of the runs of profile_commands() found under `root`;
    a summary whose runs are absent is left as it is."""
    out_dir = out_dir or PROFILES_DIR
    cal = _copy_scales(root)
    if cal is not None:
        with open(os.path.join(out_dir, "pmc_copy_calibration.txt"), "w") as fh:
            fh.write("# HBM traffic calibration (plain device copy of known size)\n")
            fh.write("commands (from the repository root, TMPDIR=/tmp):\n")
            fh.write("\n".join(_cmd_lines(("copy_fetch", "copy_write"), root)) + "\n")
            fh.write("copy: torch copy_ of %d bytes (reads %d, writes %d) -> %s, %d/%d dispatches\n"
                     % (COPY_BYTES, COPY_BYTES, COPY_BYTES, cal["kernel"], *cal["dispatches"]))
            fh.write("FETCH_SIZE_KiB_per_dispatch: %.1f   (expected %.1f) -> fetch_scale %.4f\n"
                     % (cal["fetch_kib"], COPY_BYTES / 1024.0, cal["fetch_scale"]))
            fh.write("WRITE_SIZE_KiB_per_dispatch: %.1f   (expected %.1f) -> write_scale %.4f\n"
                     % (cal["write_kib"], COPY_BYTES / 1024.0, cal["write_scale"]))
            fh.write("fetch_scale: %.4f\nwrite_scale: %.4f\n" % (cal["fetch_scale"],
                                                                 cal["write_scale"]))
        log("wrote profiles/pmc_copy_calibration.txt")
    scales = cal or _committed_scales(out_dir) or {"fetch_scale": 1.0, "write_scale": 1.0}
    for (fname, title, dims, tr, fe, wr, sqs, srcs, kernels) in SUMMARIES:
        dur = _durations(root, tr) if tr else {}
        fet = _counter(root, fe, "FETCH_SIZE") if fe else {}
        wri = _counter(root, wr, "WRITE_SIZE") if wr else {}
        if not dur and not fet:
            continue
        runs = [r for r in (tr, fe, wr) + tuple(sqs) if r]
        lines = ["# " + title, _source_line(srcs),
                 "commands (from the repository root, TMPDIR=/tmp):"] + _cmd_lines(runs, root)
        lines.append("counter scaling (pmc_copy_calibration.txt): FETCH_SIZE x %.4f, WRITE_SIZE x %.4f"
                     % (scales["fetch_scale"], scales["write_scale"]))
        if dur:
            lines += ["", "%-62s %7s %10s %10s %12s %10s" % ("kernel", "calls", "avg_us", "median_us",
                                                              "working_us", "total_ms")]
            for k, v in sorted(dur.items(), key=lambda kv: -sum(kv[1])):
                lines.append("%-62s %7d %10.3f %10.3f %12.3f %10.3f"
                             % (k[:62], len(v), np.mean(v), np.median(v), _working(v), sum(v) * 1e-3))
        for frag in kernels:
            names = sorted({k for k in list(dur) + list(fet) if frag in k})
            for k in names:
                sec = ["", "## %s, %s" % (frag, "x".join(map(str, dims))), "kernel: " + k.split("(")[0],
                       _source_line(srcs)]
                d = dur.get(k)
                if d:
                    sec.append("launches: %d, avg_us: %.3f, working_median_us: %.3f"
                               % (len(d), np.mean(d), _working(d)))
                alg = algorithmic_bytes(k, dims)
                if k in fet and k in wri:
                    fk, wk = _working(fet[k]), _working(wri[k])
                    traffic = 1024.0 * (fk * scales["fetch_scale"] + wk * scales["write_scale"])
                    sec += ["dispatches: %d (FETCH_SIZE), %d (WRITE_SIZE)" % (len(fet[k]), len(wri[k])),
                            "FETCH_SIZE_KiB_per_dispatch: %.1f" % fk,
                            "WRITE_SIZE_KiB_per_dispatch: %.1f" % wk,
                            "traffic_bytes_per_launch: %d" % round(traffic)]
                    if alg:
                        sec.append("traffic_over_algorithmic: %.3f" % (traffic / alg))
                if alg:
                    sec.append("algorithmic_bytes_per_launch: %d" % alg)
                    if d:
                        sec.append("algorithmic_GBs_at_working_median: %.1f (%.3f of %.0f)"
                                   % (alg / (_working(d) * 1e-6) / 1e9,
                                      alg / (_working(d) * 1e-6) / 1e9 / HBM_PEAK_GBS, HBM_PEAK_GBS))
                for sq in sqs:
                    rows = {}
                    for r in _csv_rows(root, sq, "counter_collection.csv"):
                        if r.get("Kernel_Name", "") == k:
                            rows.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
                    if rows:
                        sec.append("%s: %s" % (sq, ", ".join("%s=%.0f" % (c, _working(v))
                                                              for c, v in sorted(rows.items()))))
                        if "SQ_INSTS_VALU" in rows and d:
                            # one wave64 VALU instruction per CU per cycle (quarter-rate
                            # transcendentals take longer): a lower bound on VALU time
                            iss = _working(rows["SQ_INSTS_VALU"]) / 256.0 / 2400.0
                            sec.append("valu_issue_us_lower_bound: %.1f (%.2f of the working "
                                       "median)" % (iss, iss / _working(d)))
                lines += sec
        lines += ["", "reading: traffic = FETCH_SIZE and WRITE_SIZE (KiB per dispatch, the median "
                  "of the working launches) times the copy-calibrated scales; SQ_INSTS_VALU counts "
                  "wave instructions, and one CU issues about one wave64 VALU instruction per "
                  "cycle, so VALU issue alone is SQ_INSTS_VALU / 256 CUs / 2.4 GHz."]
        with open(os.path.join(out_dir, fname), "w") as fh:
            fh.write("\n".join(lines) + "\n")
        log("wrote profiles/%s" % fname)
    bt = _durations(root, "bench_trace")
    if bt:
        lines = ["# rocprofv3 kernel trace of the bench step (cantilever 96x48x48, random-field "
                 "densities, seed 1): calibration, 1 warm-up and 5 timed steps of each precision "
                 "path, product timings at 96x48x48", _source_line(PRODUCT_SOURCES),
                 "command (from the repository root, TMPDIR=/tmp):"] + _cmd_lines(("bench_trace",), root)
        lines += ["", "%-62s %7s %10s %10s %10s %7s" % ("kernel", "calls", "avg_us", "median_us",
                                                        "total_ms", "pct")]
        tot = sum(sum(v) for v in bt.values())
        for k, v in sorted(bt.items(), key=lambda kv: -sum(kv[1])):
            lines.append("%-62s %7d %10.3f %10.3f %10.3f %7.2f"
                         % (k.split("(")[0][:62], len(v), np.mean(v), np.median(v), sum(v) * 1e-3,
                            100.0 * sum(v) / tot))
        with open(os.path.join(out_dir, "kernel_trace_cantilever_96x48x48.txt"), "w") as fh:
            fh.write("\n".join(lines) + "\n")
        log("wrote profiles/kernel_trace_cantilever_96x48x48.txt")


def energy_norm_err(A, ctx, x, u, uref):
    """||u - u_ref||_K / ||u_ref||_K (Eq. 2's energy norm) with the float64
    product on ctx; both vanish on the fixed DOFs, whose identity rows then
    contribute nothing."""
    import torch
    ur = torch.as_tensor(uref, device=u.device)
    e = u - ur
    ke = A.to_matvec(ctx, x, e)
    ku = A.to_matvec(ctx, None, ur)
    return float(torch.sqrt(torch.clamp(torch.dot(e, ke), min=0.0) / torch.dot(ur, ku)).item())


def within_target(A, ctx, x, u, c, dc, ur, cr, dcr, lim=CAL_MARGIN * TARGET):
    """c, dc (2-norm) and u (energy norm) within lim of the reference."""
    return (abs(c - cr) / abs(cr) <= lim and rel2(dc.cpu().numpy(), dcr) <= lim
            and energy_norm_err(A, ctx, x, u, ur) <= lim)


class Calibrator:
    """Chooses, per request class (grid, boundary condition) and precision
    path, the loosest outer residual tolerance on RTOL_LADDER whose compliance,
    sensitivity (2-norm) and displacement (energy norm) are within TARGET of a
    float64 reference solved to 1e-11 (with a 2x margin: CAL_MARGIN), on three
    calibration seeds per class that are never timed."""

    def __init__(self, A, inputs, dev):
        self.A, self.inputs, self.dev = A, inputs, dev
        self.refs, self.cache, self.ctx = {}, {}, {}

    def field(self, dims, seed):
        import torch
        return torch.from_numpy(self.inputs.random_field(*dims, seed=seed, ell=min(6.0, dims[2] / 4),
                                                         kappa=2.0)).to(self.dev)

    def reference(self, dims, bc, seed):
        key = (dims, bc, seed)
        if key not in self.refs:
            A = self.A
            ck = (dims, bc, "ref")
            if ck not in self.ctx:
                self.ctx[ck] = A.to_create(A.Problem(*dims, bc=bc, precision=A.PREC_FP64, rtol=1e-11,
                                                     max_iters=10 ** 6))
            x = self.field(dims, seed)
            u, info, st = A.to_solve(self.ctx[ck], x, raise_on_error=False)
            assert info["rel_res"] <= 1e-10, info
            c, dc = A.to_compliance_sensitivity(self.ctx[ck], x, u)
            self.refs[key] = (u.cpu().numpy(), c, dc.cpu().numpy())
        return self.refs[key]

    def rtol(self, dims, bc, prec, seeds=None):
        key = (dims, bc, prec)
        if key in self.cache:
            return self.cache[key]
        A = self.A
        seeds = seeds or tuple(2000 + 7 * dims[0] + 3 * bc + i for i in range(3))
        chosen = RTOL_LADDER[-1]
        for rt in RTOL_LADDER:
            ctx = A.to_create(A.Problem(*dims, bc=bc, precision=prec, rtol=rt, max_iters=10 ** 6))
            ok = True
            for sd in seeds:
                x = self.field(dims, sd)
                u, info, _ = A.to_solve(ctx, x)
                c, dc = A.to_compliance_sensitivity(ctx, x, u)
                ur, cr, dcr = self.reference(dims, bc, sd)
                ok &= within_target(A, ctx, x, u, c, dc, ur, cr, dcr)
            ctx.close()
            if ok:
                chosen = rt
                break
        # the error/residual ratio varies by orders of magnitude between designs
        # of one class; the safety factor covers designs the seeds do not
        chosen = max(chosen * CAL_SAFETY, RTOL_FLOOR)
        log("calibrated %s bc=%d prec=%d: rtol %.0e" % ("x".join(map(str, dims)), bc, prec, chosen))
        self.cache[key] = chosen
        return chosen


def golden(name):
    """Values written by the oracle (tests/golden/make_bench_golden.py)."""
    meta = json.load(open(os.path.join(ROOT, "tests", "golden", name + ".json")))
    npz = os.path.join(ROOT, "tests", "golden", name + ".npz")
    arr = np.load(npz) if os.path.exists(npz) else None
    return meta, arr


def copy_rate(dev, reps=10):
    """Achievable HBM bandwidth: a device copy of COPY_BYTES (read + write)."""
    import torch
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s = torch.cuda.current_stream()
    e0.record(s)
    for _ in range(reps):
        b.copy_(a)
    e1.record(s)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * COPY_BYTES / (us * 1e-6) / 1e9


def config0(A, dev, reps=20):
    """The 24x12x6 cantilever at uniform x = 0.5: latency of the step (solve to
    1e-10, compliance and sensitivity, density filter rmin 1.5, its adjoint and
    the sensitivity filter R = 2 on dc) in both precisions, and the errors of c
    and dc against the oracle's direct solve (tests/golden)."""
    import torch
    meta, _ = golden("cantilever_24x12x6_uniform")
    dcr = np.array(meta["dc"])
    x = torch.full((24 * 12 * 6,), 0.5, dtype=torch.float64, device=dev)
    out = {"workload": "cantilever 24x12x6, x = 0.5, rtol 1e-10"}
    for name, prec in (("fp64", A.PREC_FP64), ("fp32_refine", A.PREC_FP32_REFINE)):
        ctx = A.to_create(A.Problem(24, 12, 6, precision=prec, rtol=1e-10))
        u = torch.empty(ctx.prob.ndof, dtype=torch.float64, device=dev)
        dc = torch.empty(ctx.prob.nel, dtype=torch.float64, device=dev)
        xf, g1, g2 = torch.empty_like(dc), torch.empty_like(dc), torch.empty_like(dc)
        lat = []
        for r in range(reps + 2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info, _ = A.to_solve(ctx, x, u=u)
            c, _ = A.to_compliance_sensitivity(ctx, x, u, dc=dc)
            A.to_filter(ctx, 1.5, A.FILTER_DENS, x, out=xf)
            A.to_filter(ctx, 1.5, A.FILTER_DENS_T, dc, out=g1)
            A.to_filter(ctx, 2.0, A.FILTER_SENS, dc, x=x, out=g2)
            torch.cuda.synchronize()
            if r >= 2:
                lat.append((time.perf_counter() - t0) * 1e3)
        out[name] = {"ms_p50": round(float(np.median(lat)), 4), "ms_max": round(max(lat), 4),
                     "inner_iters": info["inner_iters"], "c": c,
                     "err_vs_oracle": {"c": abs(c - meta["c"]) / abs(meta["c"]),
                                       "dc": rel2(dc.cpu().numpy(), dcr)}}
        ctx.close()
    log("config 0: %s" % out)
    return out


def main():
    args = parse()
    if args.probe:
        probe(args.probe)
        return
    if args.profile_commands:
        for cmd in profile_commands(args.profile_commands):
            print(cmd)
        return
    if args.summarize:
        summarize(args.summarize)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (independent "
              "designs would shard across GPUs with no communication). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2605_04735_amd import api as A
    from paper_2605_04735_amd import inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    nelx, nely, nelz = DIMS

    def problem(prec, rtol):
        return A.Problem(nelx, nely, nelz, precision=prec, rtol=rtol, max_iters=500000)

    def field(seed):
        return torch.from_numpy(inputs.random_field(nelx, nely, nelz, seed=seed, ell=6.0,
                                                    kappa=2.0)).to(dev)

    # ---------------------------------------------------------- calibration
    cal = Calibrator(A, inputs, dev)
    t_cal = time.perf_counter()
    rtol_mixed = cal.rtol(DIMS, A.BC_CANTILEVER, A.PREC_FP32_REFINE, seeds=(11, 12, 13))
    rtol_fp64 = cal.rtol(DIMS, A.BC_CANTILEVER, A.PREC_FP64, seeds=(11, 12, 13))
    log("calibration %.1fs: rtol mixed %.0e fp64 %.0e" % (time.perf_counter() - t_cal, rtol_mixed,
                                                           rtol_fp64))
    reference = cal.reference

    # ---------------------------------------------------------- timed steps
    x = field(1)
    uref, cref, dcref = reference(DIMS, A.BC_CANTILEVER, 1)
    prob_m = problem(A.PREC_FP32_REFINE, rtol_mixed)
    prob_d = problem(A.PREC_FP64, rtol_fp64)
    ctx_m = A.to_create(prob_m)
    ctx_d = A.to_create(prob_d)
    # the density->SDF transfer depends on x alone: it runs on a context of
    # its own, on a second stream, issued before the solve and joined at the
    # end of the step; the solve at this size leaves most of the chip idle
    # between its dependent launches
    sdf_stream = torch.cuda.Stream(device=dev)
    ctx_sdf = A.to_create(problem(A.PREC_FP64, rtol_fp64), stream=sdf_stream)
    sdf_done = torch.cuda.Event()
    nel, nn, ndof = prob_m.nel, prob_m.nn, prob_m.ndof
    f64 = dict(dtype=torch.float64, device=dev)
    bufs = dict(u=torch.empty(ndof, **f64), dc=torch.empty(nel, **f64), xf=torch.empty(nel, **f64),
                dcf=torch.empty(nel, **f64), phi=torch.empty(nn, **f64), rho=torch.empty(nn, **f64),
                vf=torch.empty(nel, **f64))

    def step(ctx):
        A.to_density_to_sdf(ctx_sdf, x, 0.5, phi=bufs["phi"], rho_nodes=bufs["rho"], vf=bufs["vf"])
        sdf_done.record(sdf_stream)
        _, info, _ = A.to_solve(ctx, x, u=bufs["u"])
        c, _ = A.to_compliance_sensitivity(ctx, x, bufs["u"], dc=bufs["dc"])
        A.to_filter(ctx, 1.5, A.FILTER_DENS, x, out=bufs["xf"])
        A.to_filter(ctx, 2.0, A.FILTER_SENS, bufs["dc"], x=x, out=bufs["dcf"])
        torch.cuda.current_stream().wait_event(sdf_done)
        return info, c

    def timed(ctx, label):
        for _ in range(args.warmup):
            step(ctx)
        torch.cuda.synchronize()
        A.to_profile(ctx, True)
        lat, iters = [], []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ts = time.perf_counter()
            info, c = step(ctx)
            torch.cuda.synchronize()  # the step's latency ends with its last result
            lat.append((time.perf_counter() - ts) * 1e3)
            iters.append(info["inner_iters"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        mv_ms, mv_n = A.to_profile(ctx, False)
        log("%s: %.2f ms/step, %d inner iterations, product %.2f us avg over %d launches"
            % (label, (t1 - t0) * 1e3 / args.steps, iters[-1], 1e3 * mv_ms / max(mv_n, 1), mv_n))
        return dict(sec=t1 - t0, lat=lat, iters=iters, info=info, c=c, mv_ms=mv_ms, mv_n=mv_n)

    res_m = timed(ctx_m, "fp32+refine")
    c_m, dc_m, u_m = res_m["c"], bufs["dc"].cpu().numpy(), bufs["u"].cpu().numpy()
    res_d = timed(ctx_d, "fp64")
    c_d, dc_d, u_d = res_d["c"], bufs["dc"].cpu().numpy(), bufs["u"].cpu().numpy()
    ntri = A.last_triangle_count(ctx_sdf)
    ctx_sdf.close()

    # ---------------------------------------------------------- products
    def product_rate(ctx, prob, f32, reps=200):
        u = torch.randn(prob.ndof, dtype=torch.float32 if f32 else torch.float64, device=dev)
        y = torch.empty_like(u)
        xx = torch.from_numpy(inputs.random_field(prob.nelx, prob.nely, prob.nelz, seed=3,
                                                  ell=6.0)).to(dev)
        mv = A.to_matvec_f32 if f32 else A.to_matvec
        mv(ctx, xx, u, y)
        for _ in range(5):
            mv(ctx, None, u, y)
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            mv(ctx, None, u, y)
        e1.record(s)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        return us, prob.ndof / (us * 1e-6) / 1e9

    copy_gbs = copy_rate(dev)
    log("device copy: %.0f GB/s" % copy_gbs)
    products = {"hbm_copy_GBs_measured": round(copy_gbs, 1), "hbm_peak_GBs_nominal": HBM_PEAK_GBS}
    us, g = product_rate(ctx_m, prob_m, True)
    products["96x48x48_f32"] = {"us": us, "gdofs": g}
    us, g = product_rate(ctx_d, prob_d, False)
    products["96x48x48_f64"] = {"us": us, "gdofs": g}
    if not args.no_large:
        for f32 in (True, False):
            pl = A.Problem(*LARGE, precision=A.PREC_FP32_REFINE if f32 else A.PREC_FP64)
            cl = A.to_create(pl)
            us, g = product_rate(cl, pl, f32, reps=50)
            kern = A.product_kernel_name(f32)
            byt = algorithmic_bytes(kern, LARGE)
            gbs = byt / (us * 1e-6) / 1e9
            products["256x128x128_%s" % ("f32" if f32 else "f64")] = {
                "us": us, "gdofs": g, "kernel": kern, "algorithmic_bytes": byt,
                "algorithmic_GBs": gbs, "frac_hbm": gbs / HBM_PEAK_GBS,
                "frac_measured_copy": gbs / copy_gbs,
                "traffic_bytes": measured_traffic("pmc_product_256x128x128.txt", "void topo::" + kern)}
            cl.close()
            del cl
            torch.cuda.empty_cache()
    for k, v in products.items():
        log("product %s: %s" % (k, v))

    # ---------------------------------------------------------- workloads
    workloads = {}
    if not args.no_large:
        workloads["mbb_sdf_ersatz_192x64x32"] = workload_mbb_sdf(A, inputs, dev, cal)
        workloads["cantilever_256x128x128"] = workload_large(A, inputs, dev, copy_gbs)
    if not args.no_simp:
        workloads["simp_cantilever_96x48x48"] = workload_simp(A, dev, rtol_mixed, rtol_fp64)
    if not args.no_levelset:
        workloads["levelset"] = workload_levelset(A, inputs, dev)
    if not args.no_paper:
        workloads["paper_problems_40x20x20"] = workload_paper(A, dev)
        workloads["levelset_iteration_40x20x20"] = workload_ls_iteration(A, dev)
    if not args.no_shape:
        workloads["shape_extension"] = workload_shape(A, inputs, dev, x,
                                                      torch.from_numpy(u_m).to(dev))

    # ---------------------------------------------------------- roofline
    # dominant kernel: the fused inner-CG product in float32.  Its HBM
    # roofline is taken at 256x128x128, where the working set (about 0.7 GB)
    # cannot stay in the caches; at the benchmark's 96x48x48 the CG working
    # set (about 30 MB) sits in the 256 MB Infinity Cache and every launch is
    # a few microseconds, so that figure (given beside it) measures launch
    # latency, not HBM.
    kern = A.cg_product_kernel_name(DIMS)
    mv_us = 1e3 * res_m["mv_ms"] / max(res_m["mv_n"], 1)
    bytes_launch = algorithmic_bytes(kern, DIMS)
    achieved = bytes_launch / (mv_us * 1e-6) / 1e9
    small = {"grid": "96x48x48", "achieved": round(achieved, 1), "frac": round(achieved / HBM_PEAK_GBS, 4),
             "avg_us": round(mv_us, 3), "bytes_per_launch": bytes_launch,
             "traffic": measured_traffic("pmc_cg_matvec_f32_cantilever_96x48x48.txt", "void topo::" + kern),
             "note": "working set resident in the Infinity Cache: launch-latency bound"}
    big = workloads.get("cantilever_256x128x128", {}).get("roofline_cg_product")
    if big is not None:
        roofline = dict(big)
        roofline["grid"] = "256x128x128 (inner-CG product inside the fp32+refine solve)"
        prof_us = profiled_avg_us(LARGE_TRACE, "void topo::" + roofline["kernel"])
        if prof_us:
            roofline["rocprofv3"] = {
                "summary": "profiles/" + LARGE_TRACE, "avg_us": prof_us,
                "achieved": round(roofline["bytes_per_launch"] / (prof_us * 1e-6) / 1e9, 1),
                "frac": round(roofline["bytes_per_launch"] / (prof_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                "note": "average over every launch of the same solve, graph replays included; "
                        "the live figure samples separate dispatches"}
        roofline["cache_resident_96x48x48"] = small
    else:
        roofline = {"bound": "hbm", "achieved": small["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": small["frac"], "traffic": small["traffic"], "kernel": kern,
                    "avg_us": small["avg_us"], "bytes_per_launch": bytes_launch, "grid": "96x48x48"}
    roofline["measured_copy_GBs"] = round(copy_gbs, 1)
    roofline["frac_of_measured_copy"] = round(roofline["achieved"] / copy_gbs, 4)

    # ---------------------------------------------------------- errors
    gmeta, garr = golden("cantilever_96x48x48_seed1")

    def errs(u, c, dc, ur, cr, dcr):
        # the energy norm with the float64 product (checked against the oracle's
        # assembled operator to 1e-13 by the parity tests)
        ut = torch.from_numpy(u).to(dev)
        return {"u": rel2(u, ur), "u_energy": energy_norm_err(A, ctx_d, x, ut, ur),
                "c": abs(c - cr) / abs(cr), "dc": rel2(dc, dcr),
                "dc_max": float(np.abs(dc - dcr).max() / np.abs(dcr).max())}
    errors = {
        "vs_oracle": {
            "fp32_refine": errs(u_m, c_m, dc_m, garr["u"], gmeta["c"], garr["dc"]),
            "fp64": errs(u_d, c_d, dc_d, garr["u"], gmeta["c"], garr["dc"]),
            "reference": "the oracle's float64 Jacobi-PCG solve of the same design to 1e-10 "
                         "(tests/golden/cantilever_96x48x48_seed1, written by "
                         "tests/golden/make_bench_golden.py)"},
        "vs_gpu_fp64_1e-11": {
            "fp32_refine": errs(u_m, c_m, dc_m, uref, cref, dcref),
            "fp64": errs(u_d, c_d, dc_d, uref, cref, dcref)}}
    log("errors vs oracle: %s" % errors["vs_oracle"])

    sps_m = args.steps / res_m["sec"]
    sps_d = args.steps / res_d["sec"]
    lat = np.array(res_m["lat"])
    out = {
        "metric": METRIC, "value": round(sps_m, 3), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * res_m["sec"] / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "cantilever 96x48x48 hex8 (698,691 DOF), random-field densities "
                               "(l=6, kappa=2, seed 1); step = fp32-inner/fp64-refined solve + "
                               "compliance/sensitivity + density and sensitivity filters + "
                               "density->SDF and vf (on a second stream, concurrent with the "
                               "solve)",
                   "rtol_fp32_refine": rtol_mixed, "rtol_fp64": rtol_fp64},
        "fp64_solves_per_s": round(sps_d, 3),
        "speedup_fp32_refine_vs_fp64": round(sps_m / sps_d, 3),
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "cg_iterations": {"fp32_refine": res_m["iters"][-1], "fp64": res_d["iters"][-1],
                          "fp32_refine_outer": res_m["info"]["outer_iters"]},
        "cg_iters_per_s": {"fp32_refine": res_m["iters"][-1] * sps_m,
                           "fp64": res_d["iters"][-1] * sps_d},
        "products": products, "errors": errors, "triangles": ntri, "roofline": roofline,
        "workloads": workloads,
    }
    if not args.no_config0:
        out["config0"] = config0(A, dev)

    # ---------------------------------------------------------- serving
    if not args.no_serving:
        out["serving"] = serving(args.requests, cal)

    # ---------------------------------------------------------- CPU oracle
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(x.cpu().numpy(), res_d["iters"][-1], ntri, args.cpu_iters)
    print(json.dumps(out), flush=True)


def _timed_solve(A, ctx, x, u=None):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, info, st = A.to_solve(ctx, x, u=u, raise_on_error=False)
    c, dc = A.to_compliance_sensitivity(ctx, x, u)
    torch.cuda.synchronize()
    return u, c, dc, info, st, (time.perf_counter() - t0) * 1e3


def workload_mbb_sdf(A, inputs, dev, cal):
    """MBB half-beam 192x64x32: SIMP-like densities (l = 6, kappa = 8, seed 2,
    shifted so that 40% of the elements exceed 0.5) -> density->SDF at 0.5 ->
    per-element volume fraction -> ersatz moduli E = max(vf, 1e-3) (penal 1,
    Emin 0) -> compliance and sensitivity, float32-inner/float64-refined and
    float64.  Each path runs at the tolerance calibrated for this workload the
    way the headline's is (the loosest ladder rung whose c, dc and energy-norm
    u errors are within half the target on three designs of the same recipe,
    seeds 21-23, times the safety factor, floored), and both also at 1e-8;
    errors against a float64 solve to 3e-10 (its stagnation floor is near
    2e-10).  The precision for this class of designs is then the path that
    solves the three calibration designs faster at its calibrated tolerance
    (`precision_choice`): on these ersatz designs float32 refinement passes
    each stop near eps32 times the condition number and every pass must
    resolve the slow modes again, so float64 in one pass can win."""
    import torch
    dims = (192, 64, 32)

    def make(geo, seed):
        x = torch.from_numpy(inputs.random_field(*dims, seed=seed, ell=6.0, kappa=8.0,
                                                 solid_fraction=0.4)).to(dev)
        _, _, vf = A.to_density_to_sdf(geo, x, 0.5)
        return torch.clamp(vf, min=1e-3)

    def problem(prec, rtol):
        return A.Problem(*dims, bc=A.BC_MBB, penal=1.0, Emin=0.0, precision=prec, rtol=rtol,
                         max_iters=10 ** 6)

    geo = A.to_create(A.Problem(*dims, bc=A.BC_MBB))
    x = torch.from_numpy(inputs.random_field(*dims, seed=2, ell=6.0, kappa=8.0,
                                             solid_fraction=0.4)).to(dev)
    A.to_density_to_sdf(geo, x, 0.5)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phi, _, vf = A.to_density_to_sdf(geo, x, 0.5)
    torch.cuda.synchronize()
    t_sdf = (time.perf_counter() - t0) * 1e3
    ntri = A.last_triangle_count(geo)
    xe = torch.clamp(vf, min=1e-3)
    out = {"sdf_ms": round(t_sdf, 3), "triangles": ntri,
           "solid_fraction_vf": float(vf.mean().item())}
    # references: float64 to 3e-10
    refc = A.to_create(problem(A.PREC_FP64, 3e-10))
    refs, designs = {}, {}
    for sd in (2, 21, 22, 23):
        designs[sd] = xe if sd == 2 else make(geo, sd)
        u, c, dc, info, st, ms = _timed_solve(A, refc, designs[sd])
        refs[sd] = (u.clone(), c, dc.cpu().numpy())
    # calibration: per precision the tolerance, then the time of each path on
    # the calibration designs at that tolerance, which picks the precision
    # for this class of designs
    rt_cal, cal_ms = {}, {}
    for name, prec in (("fp32_refine", A.PREC_FP32_REFINE), ("fp64", A.PREC_FP64)):
        chosen = RTOL_LADDER[-1]
        for rt in RTOL_LADDER:
            ctx = A.to_create(problem(prec, rt))
            ok = True
            for sd in (21, 22, 23):
                u, c, dc, _, _, _ = _timed_solve(A, ctx, designs[sd])
                ur, cr, dcr = refs[sd]
                ok &= within_target(A, ctx, designs[sd], u, c, dc, ur, cr, dcr)
            ctx.close()
            if ok:
                chosen = rt
                break
        rt_cal[name] = max(chosen * CAL_SAFETY, RTOL_FLOOR)
        ctx = A.to_create(problem(prec, rt_cal[name]))
        _timed_solve(A, ctx, designs[21])  # warm (graphs are built on first use)
        cal_ms[name] = sum(_timed_solve(A, ctx, designs[sd])[5] for sd in (21, 22, 23))
        ctx.close()
    out["rtol_calibrated"] = rt_cal
    pick = min(cal_ms, key=cal_ms.get)
    out["precision_choice"] = {
        "chosen": pick, "calibration_ms": {k: round(v, 1) for k, v in cal_ms.items()},
        "rule": "the path faster on the class's three calibration designs (seeds 21-23), each at "
                "its calibrated tolerance"}
    ur, cr, dcr = refs[2]
    for name, prec in (("fp32_refine", A.PREC_FP32_REFINE), ("fp64", A.PREC_FP64)):
        for tag, rtol in (("calibrated", rt_cal[name]), ("rtol_1e-8", 1e-8)):
            ctx = A.to_create(problem(prec, rtol))
            _timed_solve(A, ctx, xe)  # warm
            ms_all = []
            for _ in range(3):
                u, c, dc, info, st, ms = _timed_solve(A, ctx, xe)
                ms_all.append(ms)
            rec = {"rtol": rtol, "ms": round(float(np.median(ms_all)), 2),
                   "status": A.L.STATUS_NAMES.get(st, st), "inner_iters": info["inner_iters"],
                   "outer_iters": info["outer_iters"], "rel_res": info["rel_res"],
                   "err": {"u": rel2(u.cpu().numpy(), ur.cpu().numpy()),
                           "u_energy": energy_norm_err(A, ctx, xe, u, ur),
                           "c": abs(c - cr) / abs(cr), "dc": rel2(dc.cpu().numpy(), dcr)}}
            out.setdefault(name, {})[tag] = rec
            ctx.close()
    for tag in ("calibrated", "rtol_1e-8"):
        out["speedup_fp32_refine_vs_fp64_" + tag] = round(out["fp64"][tag]["ms"]
                                                          / out["fp32_refine"][tag]["ms"], 3)
    # the chosen path on the timed design, against plain float64
    out["precision_choice"]["ms"] = out[pick]["calibrated"]["ms"]
    out["precision_choice"]["speedup_vs_fp64"] = round(out["fp64"]["calibrated"]["ms"]
                                                       / out[pick]["calibrated"]["ms"], 3)
    refc.close()
    geo.close()
    log("mbb+sdf 192x64x32: sdf %.1f ms (%d triangles); fp32+refine %s; fp64 %s"
        % (t_sdf, ntri, out["fp32_refine"], out["fp64"]))
    return out


def workload_simp(A, dev, rtol_mixed, rtol_fp64, iters=12):
    """The SIMP stage on the cantilever 96x48x48: from x = V_f = 0.4, penal 3,
    sensitivity filter R = 2 (Eq. 4), OC updates (move 0.2, eta 1/2), a fixed
    number of design iterations (no Delta rho_max stop, so both precisions do
    the same work), each precision at its calibrated tolerance.  The OC update
    is also timed on its own, on the final design and its filtered
    sensitivity."""
    import torch
    dims = (96, 48, 48)
    out = {"iters": iters, "vf": 0.4, "rmin": 2.0}
    for name, prec, rtol in (("fp32_refine", A.PREC_FP32_REFINE, rtol_mixed),
                             ("fp64", A.PREC_FP64, rtol_fp64)):
        ctx = A.to_create(A.Problem(*dims, precision=prec, rtol=rtol, max_iters=10 ** 6))
        A.to_simp(ctx, vf=0.4, rmin=2.0, change_tol=0.0, max_iters=2)  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, u, info, hist, _ = A.to_simp(ctx, vf=0.4, rmin=2.0, change_tol=0.0, max_iters=iters)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        rec = {"ms_per_iter": round(ms / iters, 3), "iters_per_s": round(iters / (ms * 1e-3), 3),
               "inner_iters": info["inner_iters"], "c_first": float(hist[0]),
               "c_last": float(hist[-1]), "change_last": info["change"],
               "volume": info["volume"]}
        if name == "fp32_refine":
            _, dc = A.to_compliance_sensitivity(ctx, x, u)
            dcf = A.to_filter(ctx, 2.0, A.FILTER_SENS, dc, x=x)
            xn = torch.empty_like(x)
            A.to_oc_update(ctx, x, dcf, 0.4, xnew=xn)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(10):
                _, oi, _ = A.to_oc_update(ctx, x, dcf, 0.4, xnew=xn)
            torch.cuda.synchronize()
            rec["oc_update_ms"] = round((time.perf_counter() - t0) * 1e2, 4)
            rec["oc_bisections"] = oi["bisections"]
        out[name] = rec
        ctx.close()
    out["speedup_fp32_refine_vs_fp64"] = round(out["fp64"]["ms_per_iter"]
                                               / out["fp32_refine"]["ms_per_iter"], 3)
    log("simp 96x48x48: %s" % out)
    return out


def workload_levelset(A, inputs, dev, nsteps=40):
    """Level-set evolution (Eqs. 21-22) and reinitialisation (Eqs. 23-24) on
    the node grids of the 96x48x48 and 256x128x128 cantilevers: phi = 2.5 x the
    distance to a union of three balls, a smooth speed of both signs, CFL
    number 1/2.  Evolution: nsteps steps in one call, timed with events around
    the call (one input check and host read, then the step launches).
    Reinitialisation to max|change| < 1e-3 h.  Algorithmic bytes per node and
    step: 24 (read phi and v, write phi) and 16 (read and write phi)."""
    import torch
    out = {}
    for dims in ((96, 48, 48), (256, 128, 128)):
        nn = (dims[0] + 1) * (dims[1] + 1) * (dims[2] + 1)
        ctx = A.to_create(A.Problem(*dims))
        phi0 = torch.from_numpy(inputs.sphere_union(*dims, 5, scale=2.5)).to(dev)
        v = torch.from_numpy(inputs.smooth_speed(*dims, 7)).to(dev)
        p = phi0.clone()
        A.to_ls_advect(ctx, p, v, gamma=0.5, nsteps=2)  # warm
        p.copy_(phi0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        A.to_ls_advect(ctx, p, v, gamma=0.5, nsteps=nsteps)
        e1.record()
        torch.cuda.synchronize()
        us_adv = e0.elapsed_time(e1) * 1e3 / nsteps
        p.copy_(phi0)
        torch.cuda.synchronize()
        e0.record()
        _, steps, change, st = A.to_ls_reinit(ctx, p, gamma=0.5, tol=1e-3, max_steps=5000,
                                              raise_on_error=False)
        e1.record()
        torch.cuda.synchronize()
        ms_re = e0.elapsed_time(e1)
        us_re = ms_re * 1e3 / max(steps, 1)
        rec = {"nodes": nn, "advect_us_per_step": round(us_adv, 3),
               "advect_GBs": round(24 * nn / (us_adv * 1e-6) / 1e9, 1),
               "advect_frac_hbm": round(24 * nn / (us_adv * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
               "reinit_steps": steps, "reinit_status": A.L.STATUS_NAMES.get(st, st),
               "reinit_ms": round(ms_re, 3), "reinit_us_per_step": round(us_re, 3),
               "reinit_GBs": round(16 * nn / (us_re * 1e-6) / 1e9, 1)}
        out["%dx%dx%d" % dims] = rec
        ctx.close()
    log("levelset: %s" % out)
    return out


def workload_paper(A, dev):
    """The paper's two benchmark problems (Secs. 4.2-4.3): 40x20x20 voxels of
    a 2x1x1 domain (h = 0.05, E0 = 1, nu = 0.3), the cantilever on four
    corner supports with a disc load and the MBB with a one-element support
    strip and a half-disc load.  The SIMP stage runs from x = V_f = 0.4 (p 3,
    R = 2h, OC) to each Delta rho_max of the paper's tables, with
    float32-inner solves to 1e-6, then density->SDF of the 0.5 % design.  The
    paper's iteration counts and single-core times (its tables, stored in
    tests/golden/paper_simp_table.json) are reported beside ours as context."""
    import torch
    table = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_simp_table.json")))
    out = {}
    for bc, name in ((A.BC_CANTILEVER_CORNERS, "cantilever_corners"), (A.BC_MBB_STRIP, "mbb_strip")):
        ctx = A.to_create(A.Problem(40, 20, 20, h=0.05, bc=bc, precision=A.PREC_FP32_REFINE,
                                    rtol=1e-6, max_iters=10 ** 6))
        A.to_simp(ctx, vf=0.4, rmin=2.0, change_tol=0.0, max_iters=2)  # warm
        rows = []
        x = None
        for tol, paper_it, paper_s in zip(table["delta_rho_max"], table[name]["iterations"],
                                          table[name]["cpu_seconds"]):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, _, info, _, st = A.to_simp(ctx, vf=0.4, rmin=2.0, change_tol=tol, max_iters=2000,
                                          raise_on_error=False)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            rows.append({"delta_rho_max": tol, "iterations": info["iters"],
                         "converged": info["converged"], "seconds": round(sec, 4),
                         "c_simp": round(info["c"], 4), "volume": round(info["volume"], 5),
                         "status": A.L.STATUS_NAMES.get(st, st),
                         "paper_iterations": paper_it, "paper_cpu_seconds": paper_s})
        A.to_density_to_sdf(ctx, x, 0.5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        A.to_density_to_sdf(ctx, x, 0.5)
        torch.cuda.synchronize()
        out[name] = {"simp": rows, "sdf_ms_of_last_design": round((time.perf_counter() - t0) * 1e3, 3),
                     "triangles": A.last_triangle_count(ctx)}
        ctx.close()
    log("paper problems: %s" % out)
    return out


def workload_ls_iteration(A, dev, iters=5):
    """One iteration of the paper's level-set stage on its cantilever
    (40x20x20, h = 0.05, Sec. 4.2), chaining the built calls: ersatz weights
    vf(phi) -> moduli max(vf, 1e-3) (penal 1, Emin 0) -> float32-inner state
    solve (warm-started) -> J' and C' nodal vectors (eta = 2h) -> their two
    Hilbertian extensions (ell = 2h, rtol 1e-6) -> 10 evolution steps at CFL
    number 0.1 -> reinitialisation (CFL number 0.5, to 1e-3 h).  The stage
    starts from the SDF of the SIMP design at Delta rho_max = 1 %.  The
    optimisers' multiplier and step rules (Eqs. 11-13, 31) are not built: the
    evolution takes the objective's extended velocity as it is.  Reported: ms
    per iteration and per part, beside the paper's 10-14 s per level-set
    iteration on one CPU core (context)."""
    import torch
    h = 0.05
    dims = (40, 20, 20)
    simp = A.to_create(A.Problem(*dims, h=h, bc=A.BC_CANTILEVER_CORNERS,
                                 precision=A.PREC_FP32_REFINE, rtol=1e-6, max_iters=10 ** 6))
    x, _, _, _, _ = A.to_simp(simp, vf=0.4, rmin=2.0, change_tol=0.01, max_iters=500)
    phi, _, _ = A.to_density_to_sdf(simp, x, 0.5)
    A.to_ls_reinit(simp, phi, gamma=0.5, tol=1e-3 * h, max_steps=2000, raise_on_error=False)
    ctx = A.to_create(A.Problem(*dims, h=h, bc=A.BC_CANTILEVER_CORNERS, penal=1.0, Emin=0.0,
                                precision=A.PREC_FP32_REFINE, rtol=1e-6, max_iters=10 ** 6))
    n = ctx.prob
    VD = n.nel * h ** 3
    u = torch.zeros(n.ndof, dtype=torch.float64, device=dev)
    gJ = torch.empty(n.nn, dtype=torch.float64, device=dev)
    gC = torch.empty_like(gJ)
    vJ = torch.empty_like(gJ)
    vC = torch.empty_like(gJ)
    parts = {k: 0.0 for k in ("ersatz", "solve", "shape", "extension", "evolve", "reinit")}
    first = True
    it_total = 0
    t_all = 0.0
    stats = []
    for it in range(iters + 1):
        marks = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        vf = A.to_volume_fraction(ctx, phi)
        xe = torch.clamp(vf, min=1e-3)
        torch.cuda.synchronize()
        marks.append(time.perf_counter())
        u, sinfo, _ = A.to_solve(ctx, xe, u0=None if first else u, u=u, raise_on_error=False)
        first = False
        c, _ = A.to_compliance_sensitivity(ctx, xe, u, want_dc=False)
        marks.append(time.perf_counter())
        A.to_shape_rhs(ctx, phi, u=u, eta=2 * h, c_s=1.0, c_0=0.0, g=gJ)
        A.to_shape_rhs(ctx, phi, eta=2 * h, c_s=0.0, c_0=-1.0 / VD, g=gC)
        torch.cuda.synchronize()
        marks.append(time.perf_counter())
        _, iJ, _, _ = A.to_hilbert_extend(ctx, gJ, ell=2 * h, v=vJ, rtol=1e-6)
        _, iC, _, _ = A.to_hilbert_extend(ctx, gC, ell=2 * h, v=vC, rtol=1e-6)
        marks.append(time.perf_counter())
        A.to_ls_advect(ctx, phi, vJ, gamma=0.1, nsteps=10)
        torch.cuda.synchronize()
        marks.append(time.perf_counter())
        _, rs, _, _ = A.to_ls_reinit(ctx, phi, gamma=0.5, tol=1e-3 * h, max_steps=2000,
                                     raise_on_error=False)
        marks.append(time.perf_counter())
        if it == 0:
            continue  # warm-up iteration
        prev = t0
        for k, t in zip(parts, marks):
            parts[k] += t - prev
            prev = t
        t_all += marks[-1] - t0
        stats.append({"c": c, "inner_cg": sinfo["inner_iters"], "ext_iters": [iJ, iC],
                      "reinit_steps": rs, "volume": float(vf.mean().item())})
    out = {"iterations": iters, "ms_per_iteration": round(1e3 * t_all / iters, 3),
           "ms_per_part": {k: round(1e3 * v / iters, 3) for k, v in parts.items()},
           "per_iteration": stats, "paper_seconds_per_iteration_cpu": [10.0, 14.0]}
    ctx.close()
    simp.close()
    log("level-set iteration 40x20x20: %s" % {k: out[k] for k in ("ms_per_iteration", "ms_per_part")})
    return out


def workload_shape(A, inputs, dev, x1, u1, reps=5):
    """Relaxed shape derivative (Eqs. 15-17) and Hilbertian extension
    (Eqs. 19-20).  On the 96x48x48 cantilever the inputs are the benchmark
    design's own: phi = its density->SDF at 0.5, u its float32-refined
    displacement; on 256x128x128, phi = 2.5 x the distance to three balls and
    a seeded u.  eta = 2h, ell = 2h, extension to rtol 1e-8.  Algorithmic
    bytes of one extension CG iteration: 97 per node (apply: read p and the
    Gamma_N mask, write q; update: read x, p, r, q, write x, r, z; direction:
    read z, p, write p)."""
    import torch
    out = {}
    for dims in ((96, 48, 48), (256, 128, 128)):
        nn = (dims[0] + 1) * (dims[1] + 1) * (dims[2] + 1)
        ctx = A.to_create(A.Problem(*dims))
        if dims == DIMS:
            phi, _, _ = A.to_density_to_sdf(ctx, x1, 0.5)
            u = u1
        else:
            phi = torch.from_numpy(inputs.sphere_union(*dims, 5, scale=2.5)).to(dev)
            u = torch.from_numpy(1e-2 * inputs.random_vector(3 * nn, 5)).to(dev)
        g = A.to_shape_rhs(ctx, phi, u=u, eta=2.0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            A.to_shape_rhs(ctx, phi, u=u, eta=2.0, g=g)
        e1.record()
        torch.cuda.synchronize()
        us_rhs = e0.elapsed_time(e1) * 1e3 / reps
        band = int((g != 0).sum().item())
        v, it, rel, st = A.to_hilbert_extend(ctx, g, ell=2.0, rtol=1e-8, raise_on_error=False)
        torch.cuda.synchronize()
        e0.record()
        v, it, rel, st = A.to_hilbert_extend(ctx, g, ell=2.0, rtol=1e-8, v=v,
                                             raise_on_error=False)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        us_it = ms * 1e3 / max(it, 1)
        out["%dx%dx%d" % dims] = {
            "nodes": nn, "rhs_us": round(us_rhs, 2), "band_nodes": band,
            "extension_ms": round(ms, 3), "extension_iters": it, "extension_rel": rel,
            "extension_status": A.L.STATUS_NAMES.get(st, st),
            "us_per_iter": round(us_it, 2),
            "GBs_per_iter": round(97 * nn / (us_it * 1e-6) / 1e9, 1)}
        ctx.close()
    log("shape/extension: %s" % out)
    return out


def workload_large(A, inputs, dev, copy_gbs):
    """Cantilever 256x128x128 (12.8M DOF), random-field densities (l = 6,
    kappa = 2, seed 3): float64, float32-inner/float64-refined, and the same
    with the inner z stored in bfloat16, each to rtol 1e-8 with compliance and
    sensitivity; errors of the mixed paths against the float64 one.  The
    float32 solve also samples its inner-CG product launches (dispatch
    timestamps), which gives the product's HBM roofline at a size whose
    working set does not fit in the caches."""
    import torch
    dims = LARGE
    x = torch.from_numpy(inputs.random_field(*dims, seed=3, ell=6.0, kappa=2.0)).to(dev)
    out, res = {}, {}
    for name, prec in (("fp64", A.PREC_FP64), ("fp32_refine", A.PREC_FP32_REFINE),
                       ("fp32_refine_bf16", A.PREC_FP32_REFINE_BF16)):
        ctx = A.to_create(A.Problem(*dims, precision=prec, rtol=1e-8, max_iters=10 ** 6))
        if prec == A.PREC_FP32_REFINE:
            A.to_profile(ctx, True)
        u, c, dc, info, st, ms = _timed_solve(A, ctx, x)
        res[name] = (u.cpu().numpy(), c, dc.cpu().numpy())
        out[name] = {"ms": round(ms, 1), "status": A.L.STATUS_NAMES.get(st, st),
                     "inner_iters": info["inner_iters"], "outer_iters": info["outer_iters"],
                     "rel_res": info["rel_res"],
                     "cg_iters_per_s": round(info["inner_iters"] / (ms * 1e-3), 1),
                     "us_per_cg_iter": round(ms * 1e3 / max(info["inner_iters"], 1), 2)}
        if prec == A.PREC_FP32_REFINE:
            mv_ms, mv_n = A.to_profile(ctx, False)
            mv_us = 1e3 * mv_ms / max(mv_n, 1)
            kern = A.cg_product_kernel_name(dims)
            byt = algorithmic_bytes(kern, dims)
            ach = byt / (mv_us * 1e-6) / 1e9
            out["roofline_cg_product"] = {
                "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4),
                "frac_of_measured_copy": round(ach / copy_gbs, 4),
                "traffic": measured_traffic("kernel_trace_cg_256x128x128.txt", "void topo::" + kern),
                "kernel": kern, "avg_us": round(mv_us, 3), "launches_sampled": mv_n,
                "bytes_per_launch": byt}
            bpn = cg_iteration_bytes_f32(cg_zfuse_dims(dims))
            out["cg_algorithmic_bytes_per_node_per_iteration"] = bpn
            # the whole iteration (product and update) against the HBM roofline:
            # the per-node bytes plus the moduli's 4 B per element
            nn, nel = _nodes(dims)
            it_bytes = bpn * nn + 4 * nel
            it_gbs = it_bytes / (out[name]["us_per_cg_iter"] * 1e-6) / 1e9
            out["roofline_cg_iteration"] = {
                "bytes_per_iteration": int(it_bytes), "achieved": round(it_gbs, 1),
                "unit": "GB/s", "frac": round(it_gbs / HBM_PEAK_GBS, 4),
                "frac_of_measured_copy": round(it_gbs / copy_gbs, 4)}
        ctx.close()
        del u, dc
        torch.cuda.empty_cache()
    ud, cd, dcd = res["fp64"]
    for name in ("fp32_refine", "fp32_refine_bf16"):
        um, cm, dcm = res[name]
        out[name]["err_vs_fp64"] = {"u": rel2(um, ud), "c": abs(cm - cd) / abs(cd),
                                    "dc": rel2(dcm, dcd)}
    log("cantilever 256x128x128: fp64 %s; fp32+refine %s; bf16 z %s"
        % (out["fp64"], out["fp32_refine"], out["fp32_refine_bf16"]))
    return out


SERVE_GRIDS = [(32, 16, 16), (64, 32, 32), (96, 48, 48), (128, 64, 64)]


def serving(nreq, cal):
    """Request stream: grids uniform over SERVE_GRIDS, cantilever or MBB by a
    coin flip, random-field densities (l = min(6, nelz/4), kappa 2, seed
    1000 + k).  A closed-loop run (all requests submitted at once) gives the
    capacity; the timed run submits at Poisson arrival times (seed 4242) at
    0.75x that capacity.  The same requests are then solved one by one with
    the plain float64 path (to_solve + to_compliance_sensitivity).  Each
    path uses the tolerance calibrated for the request's class."""
    import torch
    from paper_2605_04735_amd import api as A
    from paper_2605_04735_amd import inputs
    rng = np.random.default_rng(4242)
    reqs = []
    for k in range(nreq):
        dims = SERVE_GRIDS[rng.integers(len(SERVE_GRIDS))]
        bc = A.BC_CANTILEVER if rng.uniform() < 0.5 else A.BC_MBB
        x = inputs.random_field(*dims, seed=1000 + k, ell=min(6.0, dims[2] / 4), kappa=2.0)
        reqs.append((k, dims, bc, x))
    tol_m = {(d, b): cal.rtol(d, b, A.PREC_FP32_REFINE) for d in SERVE_GRIDS for b in (0, 1)}
    tol_d = {(d, b): cal.rtol(d, b, A.PREC_FP64) for d in SERVE_GRIDS for b in (0, 1)}
    budget = 8 << 30

    def run(arrivals):
        srv = A.Server(budget, 64)
        res = {}
        t0 = time.perf_counter()
        try:
            for (k, dims, bc, x), ta in zip(reqs, arrivals):
                while time.perf_counter() - t0 < ta:
                    for r in srv.poll():
                        res[r["tag"]] = r
                    time.sleep(0.0002)
                srv.submit(A.Problem(*dims, bc=bc, precision=A.PREC_FP32_REFINE,
                                     rtol=tol_m[(dims, bc)], max_iters=500000), x, tag=k)
            assert srv.wait_idle(600000.0) == A.L.TO_OK
            for r in srv.poll():
                res[r["tag"]] = r
            t1 = time.perf_counter()
        finally:
            srv.close()
        return res, t1 - t0

    closed, t_closed = run([0.0] * nreq)
    capacity = nreq / t_closed
    lam = 0.75 * capacity
    gaps = np.random.default_rng(4242).exponential(1.0 / lam, nreq)
    arrivals = np.cumsum(gaps) - gaps[0]
    served, t_served = run(list(arrivals))
    lat = np.array([served[k]["latency_ms"] for k in range(nreq)])
    by_grid = {}
    for k, dims, bc, x in reqs:
        by_grid.setdefault("%dx%dx%d" % dims, []).append(served[k]["latency_ms"])
    lat_by_grid = {g: {"n": len(v), "p50": float(np.percentile(v, 50)),
                       "p99": float(np.percentile(v, 99)), "max": float(np.max(v))}
                   for g, v in sorted(by_grid.items())}
    ok = all(served[k]["status"] == A.L.TO_OK for k in range(nreq))
    statuses = {}
    for k in range(nreq):
        name = A.L.STATUS_NAMES.get(served[k]["status"], str(served[k]["status"]))
        statuses[name] = statuses.get(name, 0) + 1
    failed = ["%s/%s seed %d: %s" % ("x".join(map(str, reqs[k][1])), "mbb" if reqs[k][2] else "cant",
                                    1000 + k, A.L.STATUS_NAMES.get(served[k]["status"]))
              for k in range(nreq) if served[k]["status"] != A.L.TO_OK]
    log("serving: capacity %.1f solves/s, lambda %.1f/s, p50 %.1f ms p99 %.1f ms"
        % (capacity, lam, np.percentile(lat, 50), np.percentile(lat, 99)))
    # plain float64, one request at a time, same requests
    dev = torch.device("cuda:0")
    ctxs = {}
    t0 = time.perf_counter()
    ref = {}
    for k, dims, bc, x in reqs:
        key = (dims, bc)
        if key not in ctxs:
            ctxs[key] = A.to_create(A.Problem(*dims, bc=bc, precision=A.PREC_FP64,
                                              rtol=tol_d[key], max_iters=500000))
        xg = torch.from_numpy(x).to(dev)
        u, _, _ = A.to_solve(ctxs[key], xg)
        c, dc = A.to_compliance_sensitivity(ctxs[key], xg, u)
        ref[k] = (c, dc)
    torch.cuda.synchronize()
    t_fp64 = time.perf_counter() - t0
    # errors of a sample of served and float64 results against tight references
    errs = {"served_c": 0.0, "served_dc": 0.0, "fp64_c": 0.0, "fp64_dc": 0.0}
    for k, dims, bc, x in reqs[:32]:
        seed = 1000 + k
        _, cr, dcr = tight_reference(cal, dims, bc, x)
        errs["served_c"] = max(errs["served_c"], abs(served[k]["c"] - cr) / abs(cr))
        errs["served_dc"] = max(errs["served_dc"], rel2(served[k]["dc"], dcr))
        errs["fp64_c"] = max(errs["fp64_c"], abs(ref[k][0] - cr) / abs(cr))
        errs["fp64_dc"] = max(errs["fp64_dc"], rel2(ref[k][1].cpu().numpy(), dcr))
    sps = nreq / t_served
    log("serving: capacity %.1f solves/s (served at lambda: %.1f) vs %.1f solves/s plain fp64"
        % (capacity, sps, nreq / t_fp64))
    return {"requests": nreq, "grids": ["%dx%dx%d" % g for g in SERVE_GRIDS],
            "all_ok": ok, "statuses": statuses, "failed": failed[:8],
            "capacity_closed_loop_solves_per_s": round(capacity, 2),
            "lambda_per_s": round(lam, 2), "solves_per_s": round(sps, 2),
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "max": float(lat.max())},
            "latency_ms_by_grid": lat_by_grid,
            "fp64_sequential_solves_per_s": round(nreq / t_fp64, 2),
            # the served form at saturation against plain float64; at lambda
            # (0.75x capacity) the served rate is the arrival rate by design
            "speedup_capacity_vs_fp64_sequential": round(capacity * t_fp64 / nreq, 3),
            "served_rate_at_lambda_over_fp64_sequential": round(sps * t_fp64 / nreq, 3),
            "max_rel_err_vs_tight_fp64_first32": errs,
            "rtol_served": {"%dx%dx%d/%s" % (*d, "mbb" if b else "cant"): v for (d, b), v in tol_m.items()},
            "rtol_fp64": {"%dx%dx%d/%s" % (*d, "mbb" if b else "cant"): v for (d, b), v in tol_d.items()}}


def tight_reference(cal, dims, bc, x):
    import torch
    A = cal.A
    ck = (dims, bc, "ref")
    if ck not in cal.ctx:
        cal.ctx[ck] = A.to_create(A.Problem(*dims, bc=bc, precision=A.PREC_FP64, rtol=1e-11,
                                            max_iters=10 ** 6))
    xg = torch.from_numpy(x).to(cal.dev)
    u, info, _ = A.to_solve(cal.ctx[ck], xg, raise_on_error=False)
    c, dc = A.to_compliance_sensitivity(cal.ctx[ck], xg, u)
    return None, c, dc.cpu().numpy()


def cpu_baseline(x, n_iters, ntri, cpu_iters):
    """The oracle, single-threaded, on a bounded sample of the same step, in
    two legs.  Measured: assembly of K, `cpu_iters` Jacobi-PCG iterations
    (their time per iteration extrapolated to the float64 GPU iteration count
    of the same algorithm), the sensitivity and both filters on the full grid.
    Extrapolated: the brute-force density->SDF (all nodes against all
    triangles) on a 24x12x12 crop, scaled by nodes x triangles to the full
    grid.  `value` is the whole step; `value_solve_sens_filters` leaves the
    SDF leg out."""
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(1)
    except Exception:
        limiter = None
    from oracle import element, fem, filters, sdf
    nelx, nely, nelz = DIMS
    t = time.perf_counter()
    K0 = element.k0(0.3, 1.0)
    E = fem.modulus(x, 1.0, 1e-9, 3.0)
    K = fem.assemble(nelx, nely, nelz, E, K0)
    fixed, f = fem.problem_arrays(nelx, nely, nelz, 0)
    t_asm = time.perf_counter() - t
    t = time.perf_counter()
    u, it, _ = fem.solve_pcg(K, f, fixed, rtol=1e-30, maxit=cpu_iters)
    t_pcg = (time.perf_counter() - t) / max(it, 1)
    t = time.perf_counter()
    s = fem.element_energy(nelx, nely, nelz, K0, u)
    dc = fem.sensitivity(x, s, 1.0, 1e-9, 3.0)
    filters.density_filter(x, nelx, nely, nelz, 1.5)
    filters.sensitivity_filter(x, dc, nelx, nely, nelz, 2.0)
    t_post = time.perf_counter() - t
    cx, cy, cz = 24, 12, 12
    xc = x.reshape(nelz, nely, nelx)[:cz, :cy, :cx].ravel()
    t = time.perf_counter()
    _, _, _, Tc, _ = sdf.density_to_sdf(xc, cx, cy, cz, 1.0, 0.5)
    t_sdf_crop = time.perf_counter() - t
    nn_full = (nelx + 1) * (nely + 1) * (nelz + 1)
    nn_crop = (cx + 1) * (cy + 1) * (cz + 1)
    scale = (nn_full * max(ntri, 1)) / (nn_crop * max(len(Tc), 1))
    t_sdf = t_sdf_crop * scale
    t_solve = t_asm + n_iters * t_pcg
    measured = t_asm + it * t_pcg + t_post + t_sdf_crop
    if limiter is not None:
        limiter.unregister() if hasattr(limiter, "unregister") else None
    return {"value": 1.0 / (t_solve + t_post + t_sdf), "unit": "solves/s", "cores": 1,
            "kind": "oracle",
            "value_solve_sens_filters": 1.0 / (t_solve + t_post),
            "legs_s": {"assembly": round(t_asm, 3), "pcg_per_iteration": round(t_pcg, 5),
                       "solve_extrapolated": round(t_solve, 2),
                       "sensitivity_and_filters": round(t_post, 3),
                       "sdf_crop_measured": round(t_sdf_crop, 3),
                       "sdf_extrapolated": round(t_sdf, 1)},
            "cpu_seconds_measured": round(measured, 2),
            "sample": ("96x48x48, one thread. Measured: assembly %.2fs, %d PCG iterations at "
                       "%.4fs each, sensitivity and both filters %.2fs (full grid), brute-force "
                       "SDF of a 24x12x12 crop %.2fs. Extrapolated: the solve to %d iterations "
                       "(the float64 GPU count of the same algorithm) = %.0fs; the SDF by nodes x "
                       "triangles (%d) to %.0fs"
                       % (t_asm, it, t_pcg, t_post, t_sdf_crop, n_iters, t_solve, ntri, t_sdf)),
            "host": platform.processor() or platform.machine(), "os_cpu_count": os.cpu_count()}


if __name__ == "__main__":
    main()
