"""The density -> SDF call that allocates nothing (to_density_to_sdf_noalloc)
against the one that grows its own triangle buffer, through the C ABI: the
same nodal densities, triangle count, signed distances and volume fractions,
bit for bit, on two calls in a row (the second on a smaller grid, whose
triangles overwrite a prefix of the first call's), and a clear error for a
design with more triangles than the fixed array holds."""
import numpy as np
import pytest
import torch

from paper_2605_04735_amd import api as A
from paper_2605_04735_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _both(dims, x):
    ctx = A.to_create(A.Problem(*dims))
    p = ctx.prob
    xg = torch.from_numpy(x).to(DEV)
    phi, rho, vf = A.to_density_to_sdf(ctx, xg, 0.5)
    n_ref = A.last_triangle_count(ctx)
    phi2 = torch.full((p.nn,), 7.0, dtype=torch.float64, device=DEV)
    rho2 = torch.full((p.nn,), 7.0, dtype=torch.float64, device=DEV)
    vf2 = torch.full((p.nel,), 7.0, dtype=torch.float64, device=DEV)
    A.to_density_to_sdf_noalloc(ctx, xg, phi2, rho2, vf2)
    torch.cuda.synchronize()
    assert A.last_triangle_count(ctx) == n_ref
    assert torch.equal(phi, phi2) and torch.equal(rho, rho2) and torch.equal(vf, vf2)
    return n_ref


def test_noalloc_equals_allocating_call_twice():
    print("noalloc 48x24x24 then 20x10x10", flush=True)
    big = (48, 24, 24)
    n1 = _both(big, inputs.random_field(*big, seed=21, ell=2.0, kappa=2.0))
    small = (20, 10, 10)
    n2 = _both(small, inputs.random_field(*small, seed=22, ell=2.0, kappa=2.0))
    assert 0 < n2 < n1 <= A.NOALLOC_TRI_MAX
    print("triangles %d then %d" % (n1, n2), flush=True)


def test_noalloc_rejects_too_many_triangles():
    dims = (72, 72, 64)
    print("noalloc over the cap", dims, flush=True)
    x = inputs.random_field(*dims, seed=23, ell=1.0, kappa=2.0)
    ctx = A.to_create(A.Problem(*dims))
    p = ctx.prob
    xg = torch.from_numpy(x).to(DEV)
    phi = torch.zeros(p.nn, dtype=torch.float64, device=DEV)
    st = A.to_density_to_sdf_noalloc(ctx, xg, phi, raise_on_error=False)
    n = A.last_triangle_count(ctx)
    print("triangles %d, status %d" % (n, st), flush=True)
    assert n > A.NOALLOC_TRI_MAX
    assert st == A.L.TO_E_OOM
    assert "at most" in A.L.lib().to_last_error(ctx.handle).decode()
    # phi untouched, the context still usable
    assert torch.count_nonzero(phi).item() == 0
    A.to_density_to_sdf(ctx, xg, 0.5, phi=phi)
    torch.cuda.synchronize()
    assert A.last_triangle_count(ctx) == n
