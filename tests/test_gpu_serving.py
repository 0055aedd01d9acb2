"""GPU tests of the continuous-batching server: every result is the same
alone and in a mix of concurrently served designs of different sizes and
boundary conditions; admission waits for HBM budget; results match the
single-design path and the oracle."""
import time

import numpy as np
import pytest
import torch

from oracle import element, fem
from paper_2605_04735_amd import api as A
from paper_2605_04735_amd import inputs

pytestmark = pytest.mark.gpu

MIX = [((24, 12, 8), A.BC_CANTILEVER), ((16, 8, 8), A.BC_MBB), ((32, 16, 12), A.BC_MBB),
       ((20, 10, 10), A.BC_CANTILEVER), ((12, 12, 6), A.BC_MBB), ((28, 14, 10), A.BC_CANTILEVER),
       ((20, 10, 10), A.BC_CANTILEVER_CORNERS), ((16, 8, 8), A.BC_MBB_STRIP)]


def _requests():
    reqs = []
    for k, (dims, bc) in enumerate(MIX):
        x = inputs.random_field(*dims, seed=1000 + k, ell=min(6.0, dims[2] / 4), kappa=2.0)
        prob = A.Problem(*dims, bc=bc, precision=A.PREC_FP32_REFINE, rtol=1e-6)
        reqs.append((k, prob, x))
    return reqs


def _serve(reqs, budget=1 << 30, slots=16, gap_s=0.0):
    srv = A.Server(budget, slots)
    out = {}
    try:
        for k, prob, x in reqs:
            srv.submit(prob, x, tag=k)
            if gap_s:
                time.sleep(gap_s)
        assert srv.wait_idle(300000.0) == A.L.TO_OK
        for r in srv.poll():
            out[r["tag"]] = r
    finally:
        srv.close()
    return out


def test_alone_equals_mixed_and_single_design_path():
    reqs = _requests()
    print("serving mix", len(reqs), flush=True)
    mixed = _serve(reqs)
    assert sorted(mixed) == [k for k, _, _ in reqs]
    for k, prob, x in reqs:
        alone = _serve([(k, prob, x)])[k]
        m = mixed[k]
        assert m["status"] == A.L.TO_OK and alone["status"] == A.L.TO_OK
        # bit-identical by construction; asserted within the path's tolerance
        assert abs(m["c"] - alone["c"]) <= 1e-12 * abs(alone["c"])
        assert np.max(np.abs(m["dc"] - alone["dc"])) <= 1e-12 * np.abs(alone["dc"]).max()
        print("tag", k, "identical:", m["c"] == alone["c"] and np.array_equal(m["dc"], alone["dc"]))
        # the single-design C-ABI path computes the same
        ctx = A.to_create(prob)
        xg = torch.from_numpy(x).cuda()
        u, info, _ = A.to_solve(ctx, xg)
        c, dc = A.to_compliance_sensitivity(ctx, xg, u)
        assert abs(c - m["c"]) <= 1e-12 * abs(c)
        assert np.max(np.abs(dc.cpu().numpy() - m["dc"])) <= 1e-12 * np.abs(m["dc"]).max()


def test_serving_grid_sizes_equal_single_design_path():
    """One request of each grid size of the benchmark's request stream
    (32 x 16 x 16 up to 128 x 64 x 64, cantilever and MBB alternating),
    served together: each result equals the single-design C-ABI path."""
    reqs = []
    for k, dims in enumerate([(32, 16, 16), (64, 32, 32), (96, 48, 48), (128, 64, 64)]):
        bc = A.BC_CANTILEVER if k % 2 == 0 else A.BC_MBB
        x = inputs.random_field(*dims, seed=1000 + k, ell=min(6.0, dims[2] / 4), kappa=2.0)
        reqs.append((k, A.Problem(*dims, bc=bc, precision=A.PREC_FP32_REFINE, rtol=1e-6), x))
    print("serving grid sizes", flush=True)
    served = _serve(reqs)
    for k, prob, x in reqs:
        m = served[k]
        assert m["status"] == A.L.TO_OK
        ctx = A.to_create(prob)
        xg = torch.from_numpy(x).cuda()
        u, info, _ = A.to_solve(ctx, xg)
        c, dc = A.to_compliance_sensitivity(ctx, xg, u)
        assert abs(c - m["c"]) <= 1e-12 * abs(c)
        assert np.max(np.abs(dc.cpu().numpy() - m["dc"])) <= 1e-12 * np.abs(m["dc"]).max()
        print("tag", k, (prob.nelx, prob.nely, prob.nelz), "identical:",
              c == m["c"] and np.array_equal(dc.cpu().numpy(), m["dc"]), flush=True)


def test_served_results_match_oracle():
    k, prob, x = _requests()[1]
    r = _serve([(k, prob, x)])[k]
    K0 = element.k0(0.3, 1.0)
    K = fem.assemble(prob.nelx, prob.nely, prob.nelz, fem.modulus(x, 1.0, 1e-9, 3.0), K0)
    fixed, f = fem.problem_arrays(prob.nelx, prob.nely, prob.nelz, prob.bc)
    u = fem.solve_direct(K, f, fixed)
    c = fem.compliance(f, u)
    dc = fem.sensitivity(x, fem.element_energy(prob.nelx, prob.nely, prob.nelz, K0, u), 1.0, 1e-9, 3.0)
    assert abs(r["c"] - c) <= 1e-6 * abs(c)
    assert np.linalg.norm(r["dc"] - dc) <= 1e-6 * np.linalg.norm(dc)


def test_tiny_budget_queues_and_still_finishes():
    reqs = _requests()
    big = max(reqs, key=lambda t: t[1].nel)
    # room for about one large request at a time: the rest wait in the queue
    foot = A.to_workspace_size(big[1])
    srv = A.Server(int(foot * 1.5), 8)
    try:
        for k, prob, x in reqs:
            srv.submit(prob, x, tag=k)
        st = srv.stats()
        assert st["queued"] + st["live"] >= 1
        assert srv.wait_idle(300000.0) == A.L.TO_OK
        res = {r["tag"]: r for r in srv.poll()}
    finally:
        srv.close()
    ref = _serve(reqs)
    for k, _, _ in reqs:
        assert res[k]["status"] == A.L.TO_OK
        assert res[k]["c"] == ref[k]["c"] and np.array_equal(res[k]["dc"], ref[k]["dc"])


def test_server_rejects_bad_requests():
    srv = A.Server(64 << 20, 2)
    try:
        p = A.Problem(8, 4, 4, precision=A.PREC_FP64)
        with pytest.raises(A.TopoError):
            srv.submit(p, np.full(p.nel, 0.5), tag=1)
        p = A.Problem(128, 64, 64, precision=A.PREC_FP32_REFINE)     # footprint ~100 MB > 64 MiB
        with pytest.raises(A.TopoError) as e:
            srv.submit(p, np.full(p.nel, 0.5), tag=2)
        assert e.value.status == A.L.TO_E_OOM
        p = A.Problem(8, 4, 4, precision=A.PREC_FP32_REFINE)
        bad = np.full(p.nel, 0.5)
        bad[3] = np.nan
        srv.submit(p, bad, tag=3)
        assert srv.wait_idle(60000.0) == A.L.TO_OK
        r = srv.poll()
        assert len(r) == 1 and r[0]["status"] == A.L.TO_E_NONFINITE
    finally:
        srv.close()


def test_served_graph_replays_equal_separate_launches(monkeypatch):
    """The server's chunks replayed as graphs (once a batch is stable) give
    bit-for-bit the results of separate launches."""
    reqs = _requests()
    print("serving mix with and without graphs", flush=True)
    monkeypatch.setenv("TOPO_GRAPH", "0")
    eager = _serve(reqs)
    monkeypatch.setenv("TOPO_GRAPH", "1")
    graph = _serve(reqs)
    for k, _, _ in reqs:
        assert eager[k]["status"] == A.L.TO_OK and graph[k]["status"] == A.L.TO_OK
        assert graph[k]["c"] == eager[k]["c"]
        assert np.array_equal(graph[k]["dc"], eager[k]["dc"])


def test_served_z_formed_in_product_equals_z_stored(monkeypatch):
    """The batched CG product reads each design's z source from its
    descriptor; forming z = D r there gives the stored-z results bit for bit."""
    reqs = _requests()
    print("serving mix with z stored and z formed", flush=True)
    monkeypatch.setenv("TOPO_CG_ZFUSE", "0")
    stored = _serve(reqs)
    monkeypatch.setenv("TOPO_CG_ZFUSE", "1")
    formed = _serve(reqs)
    for k, _, _ in reqs:
        assert stored[k]["status"] == A.L.TO_OK and formed[k]["status"] == A.L.TO_OK
        assert formed[k]["c"] == stored[k]["c"]
        assert np.array_equal(formed[k]["dc"], stored[k]["dc"])
