"""Python binding of the C ABI with the same call names.

Argument marshalling only: torch tensors supply device memory and the current
HIP stream; every step of the computation runs in the HIP library.
"""
import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

from . import _lib as L
from ._lib import (BC_CANTILEVER, BC_MBB, BC_CUSTOM, BC_CANTILEVER_CORNERS,  # noqa: F401
                   BC_MBB_STRIP, PREC_FP64, PREC_FP32_REFINE, PREC_FP32_REFINE_BF16,
                   FILTER_DENS, FILTER_DENS_T, FILTER_SENS)


class TopoError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (L.STATUS_NAMES.get(status, status), message))
        self.status = status
        self.message = message


@dataclass
class Problem:
    nelx: int
    nely: int
    nelz: int
    h: float = 1.0
    E0: float = 1.0
    Emin: float = 1e-9
    nu: float = 0.3
    penal: float = 3.0
    bc: int = L.BC_CANTILEVER
    fixed_mask: Optional[np.ndarray] = None   # CUSTOM: (ndof,) bool/uint8
    load: Optional[np.ndarray] = None         # CUSTOM: (ndof,) float64
    load_total: float = 1.0
    precision: int = L.PREC_FP64
    rtol: float = 1e-8
    max_iters: int = 200000
    _keep: list = field(default_factory=list, repr=False)

    @property
    def nel(self):
        return self.nelx * self.nely * self.nelz

    @property
    def nn(self):
        return (self.nelx + 1) * (self.nely + 1) * (self.nelz + 1)

    @property
    def ndof(self):
        return 3 * self.nn

    def to_c(self):
        p = L.ToProblem()
        for name in ("nelx", "nely", "nelz", "bc", "precision", "max_iters"):
            setattr(p, name, int(getattr(self, name)))
        for name in ("h", "E0", "Emin", "nu", "penal", "load_total", "rtol"):
            setattr(p, name, float(getattr(self, name)))
        self._keep = []
        if self.bc == L.BC_CUSTOM and self.fixed_mask is not None and self.load is not None:
            m = np.ascontiguousarray(np.asarray(self.fixed_mask).astype(np.uint8).ravel())
            f = np.ascontiguousarray(np.asarray(self.load, dtype=np.float64).ravel())
            if m.size != self.ndof or f.size != self.ndof:
                raise ValueError("CUSTOM mask/load must have ndof entries")
            self._keep = [m, f]
            p.fixed_mask = m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
            p.load = f.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        return p


def _err(ctx_handle=None):
    msg = L.lib().to_last_error(ctx_handle)
    return msg.decode() if msg else ""


def _check(status, ctx_handle=None):
    if status != L.TO_OK:
        raise TopoError(status, _err(ctx_handle))


def _dev(t, dtype, numel, name):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != numel:
        raise TypeError("%s must be a contiguous %s tensor with %d elements" % (name, dtype, numel))
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def to_workspace_size(prob: Problem) -> int:
    n = ctypes.c_size_t(0)
    cp = prob.to_c()
    _check(L.lib().to_workspace_size(ctypes.byref(cp), ctypes.byref(n)))
    return n.value


class Context:
    """Owns the opaque to_ctx and (when the binding allocated it) the
    workspace tensor."""

    def __init__(self, prob: Problem, workspace=None, stream=None, device="cuda"):
        self.prob = prob
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        nbytes = to_workspace_size(prob)
        if workspace is None:
            workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        ptr = workspace.data_ptr()
        aligned = (ptr + 255) & ~255
        self.workspace = workspace
        self.ws_bytes = nbytes
        h = ctypes.c_void_p(0)
        cp = prob.to_c()
        _check(L.lib().to_create(ctypes.byref(cp), ctypes.c_void_p(aligned),
                                 ctypes.c_size_t(workspace.numel() - (aligned - ptr)),
                                 _stream(self.stream), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            L.lib().to_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def last_error(self):
        return _err(self.handle)


def to_create(prob: Problem, workspace=None, stream=None) -> Context:
    return Context(prob, workspace, stream)


def to_destroy(ctx: Context):
    ctx.close()


def to_solve(ctx: Context, x, u0=None, u=None, raise_on_error=True):
    """Returns (u, info, status)."""
    p = ctx.prob
    if u is None:
        u = torch.empty(p.ndof, dtype=torch.float64, device=x.device)
    info = L.ToSolveInfo()
    st = L.lib().to_solve(ctx.handle, _dev(x, torch.float64, p.nel, "x"),
                          _dev(u0, torch.float64, p.ndof, "u0"), _dev(u, torch.float64, p.ndof, "u"),
                          ctypes.byref(info))
    if raise_on_error:
        _check(st, ctx.handle)
    return u, {"outer_iters": info.outer_iters, "inner_iters": info.inner_iters,
               "rel_res": info.rel_res, "ms": info.ms}, st


def to_compliance_sensitivity(ctx: Context, x, u, dc=None, want_dc=True):
    """Returns (c, dc)."""
    p = ctx.prob
    if dc is None and want_dc:
        dc = torch.empty(p.nel, dtype=torch.float64, device=x.device)
    c = ctypes.c_double(0.0)
    _check(L.lib().to_compliance_sensitivity(ctx.handle, _dev(x, torch.float64, p.nel, "x"),
                                             _dev(u, torch.float64, p.ndof, "u"), ctypes.byref(c),
                                             _dev(dc, torch.float64, p.nel, "dc")), ctx.handle)
    return c.value, dc


def last_energy_sum(ctx: Context) -> float:
    return L.lib().to_last_energy_sum(ctx.handle)


def to_filter(ctx: Context, rmin, mode, inp, x=None, out=None):
    p = ctx.prob
    if out is None:
        out = torch.empty(p.nel, dtype=torch.float64, device=inp.device)
    _check(L.lib().to_filter(ctx.handle, float(rmin), int(mode), _dev(x, torch.float64, p.nel, "x"),
                             _dev(inp, torch.float64, p.nel, "in"),
                             _dev(out, torch.float64, p.nel, "out")), ctx.handle)
    return out


def to_density_to_sdf(ctx: Context, x, rho_t=0.5, phi=None, rho_nodes=None, vf=None,
                      want_rho=True, want_vf=True):
    """Returns (phi, rho_nodes, vf)."""
    p = ctx.prob
    dev = x.device
    if phi is None:
        phi = torch.empty(p.nn, dtype=torch.float64, device=dev)
    if rho_nodes is None and want_rho:
        rho_nodes = torch.empty(p.nn, dtype=torch.float64, device=dev)
    if vf is None and want_vf:
        vf = torch.empty(p.nel, dtype=torch.float64, device=dev)
    _check(L.lib().to_density_to_sdf(ctx.handle, _dev(x, torch.float64, p.nel, "x"), float(rho_t),
                                     _dev(phi, torch.float64, p.nn, "phi"),
                                     _dev(rho_nodes, torch.float64, p.nn, "rho_nodes"),
                                     _dev(vf, torch.float64, p.nel, "vf")), ctx.handle)
    return phi, rho_nodes, vf


def to_density_to_sdf_noalloc(ctx: Context, x, phi, rho_nodes=None, vf=None, rho_t=0.5,
                              raise_on_error=True):
    """to_density_to_sdf without any device allocation: the triangles go to
    the library's fixed device array (at most NOALLOC_TRI_MAX of them).  The
    caller passes every output buffer.  Returns the status."""
    p = ctx.prob
    st = L.lib().to_density_to_sdf_noalloc(ctx.handle, _dev(x, torch.float64, p.nel, "x"),
                                           float(rho_t), _dev(phi, torch.float64, p.nn, "phi"),
                                           _dev(rho_nodes, torch.float64, p.nn, "rho_nodes"),
                                           _dev(vf, torch.float64, p.nel, "vf"))
    if raise_on_error:
        _check(st, ctx.handle)
    return st


NOALLOC_TRI_MAX = 262144  # TO_NOALLOC_MAX_TRIANGLES of include/to.h


def last_triangle_count(ctx: Context) -> int:
    return L.lib().to_last_triangle_count(ctx.handle)


def to_volume_fraction(ctx: Context, phi, vf=None):
    """Per-element solid volume fraction of a nodal level set; returns vf."""
    p = ctx.prob
    if vf is None:
        vf = torch.empty(p.nel, dtype=torch.float64, device=phi.device)
    _check(L.lib().to_volume_fraction(ctx.handle, _dev(phi, torch.float64, p.nn, "phi"),
                                      _dev(vf, torch.float64, p.nel, "vf")), ctx.handle)
    return vf


def to_oc_update(ctx: Context, x, dc, vf, move=0.2, eta=0.5, xnew=None, raise_on_error=True):
    """Returns (xnew, info, status); xnew may be x itself (in place)."""
    p = ctx.prob
    if xnew is None:
        xnew = torch.empty(p.nel, dtype=torch.float64, device=x.device)
    info = L.ToOcInfo()
    st = L.lib().to_oc_update(ctx.handle, _dev(x, torch.float64, p.nel, "x"),
                              _dev(dc, torch.float64, p.nel, "dc"), float(vf), float(move),
                              float(eta), _dev(xnew, torch.float64, p.nel, "xnew"),
                              ctypes.byref(info))
    if raise_on_error:
        _check(st, ctx.handle)
    return xnew, {"lambda": info.lambda_, "change": info.change, "volume": info.volume,
                  "bisections": info.bisections}, st


def to_simp(ctx: Context, vf=0.4, rmin=2.0, move=0.2, eta=0.5, change_tol=0.01, max_iters=100,
            x=None, u=None, work=None, init_uniform=None, raise_on_error=True):
    """The SIMP loop.  x: start design (None: uniform vf); it is updated in
    place.  Returns (x, u, info, c_history, status)."""
    p = ctx.prob
    dev = torch.device("cuda")
    if init_uniform is None:
        init_uniform = x is None
    if x is None:
        x = torch.empty(p.nel, dtype=torch.float64, device=dev)
    if u is None:
        u = torch.empty(p.ndof, dtype=torch.float64, device=x.device)
    if work is None:
        work = torch.empty(2 * p.nel, dtype=torch.float64, device=x.device)
    hist = np.zeros(int(max_iters), dtype=np.float64)
    sp = L.ToSimpParams(float(vf), float(rmin), float(move), float(eta), float(change_tol),
                        int(max_iters), int(bool(init_uniform)))
    info = L.ToSimpInfo()
    st = L.lib().to_simp(ctx.handle, ctypes.byref(sp), _dev(x, torch.float64, p.nel, "x"),
                         _dev(u, torch.float64, p.ndof, "u"),
                         _dev(work, torch.float64, 2 * p.nel, "work"),
                         ctypes.c_void_p(hist.ctypes.data), ctypes.byref(info))
    if raise_on_error:
        _check(st, ctx.handle)
    out = {"iters": info.iters, "converged": bool(info.converged),
           "inner_iters": info.inner_iters, "c": info.c, "change": info.change,
           "volume": info.volume, "ms": info.ms}
    return x, u, out, hist[:info.iters].copy(), st


def to_ls_advect(ctx: Context, phi, v, gamma=0.5, nsteps=1, raise_on_error=True):
    """Evolves phi in place.  Returns (phi, dt, status)."""
    p = ctx.prob
    dt = ctypes.c_double(0.0)
    st = L.lib().to_ls_advect(ctx.handle, _dev(phi, torch.float64, p.nn, "phi"),
                              _dev(v, torch.float64, p.nn, "v"), float(gamma), int(nsteps),
                              ctypes.byref(dt))
    if raise_on_error:
        _check(st, ctx.handle)
    return phi, dt.value, st


def to_ls_reinit(ctx: Context, phi, gamma=0.5, tol=1e-3, max_steps=1000, raise_on_error=True):
    """Reinitialises phi in place.  Returns (phi, steps, last change, status)."""
    p = ctx.prob
    steps = ctypes.c_int32(0)
    change = ctypes.c_double(0.0)
    st = L.lib().to_ls_reinit(ctx.handle, _dev(phi, torch.float64, p.nn, "phi"), float(gamma),
                              float(tol), int(max_steps), ctypes.byref(steps),
                              ctypes.byref(change))
    if raise_on_error:
        _check(st, ctx.handle)
    return phi, steps.value, change.value, st


def to_shape_rhs(ctx: Context, phi, u=None, eta=2.0, c_s=1.0, c_0=0.0, g=None):
    """Nodal relaxed shape-derivative vector; returns g."""
    p = ctx.prob
    if g is None:
        g = torch.empty(p.nn, dtype=torch.float64, device=phi.device)
    _check(L.lib().to_shape_rhs(ctx.handle, _dev(u, torch.float64, p.ndof, "u"),
                                _dev(phi, torch.float64, p.nn, "phi"), float(eta), float(c_s),
                                float(c_0), _dev(g, torch.float64, p.nn, "g")), ctx.handle)
    return g


def to_hilbert_extend(ctx: Context, g, ell=1.0, v=None, rtol=1e-8, max_iters=10000,
                      raise_on_error=True):
    """Returns (v, iterations, relative residual, status)."""
    p = ctx.prob
    if v is None:
        v = torch.empty(p.nn, dtype=torch.float64, device=g.device)
    it = ctypes.c_int32(0)
    rel = ctypes.c_double(0.0)
    st = L.lib().to_hilbert_extend(ctx.handle, float(ell), _dev(g, torch.float64, p.nn, "g"),
                                   _dev(v, torch.float64, p.nn, "v"), float(rtol), int(max_iters),
                                   ctypes.byref(it), ctypes.byref(rel))
    if raise_on_error:
        _check(st, ctx.handle)
    return v, it.value, rel.value, st


def to_profile(ctx: Context, enable: bool):
    """(ms, count) of inner-CG product launches since the previous call."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(L.lib().to_profile(ctx.handle, int(enable), ctypes.byref(ms), ctypes.byref(n)), ctx.handle)
    return ms.value, n.value


def to_matvec(ctx: Context, x, u, y=None):
    """x = None reuses the moduli of the previous product on ctx."""
    p = ctx.prob
    if y is None:
        y = torch.empty(p.ndof, dtype=torch.float64, device=u.device)
    _check(L.lib().to_matvec(ctx.handle, _dev(x, torch.float64, p.nel, "x"),
                             _dev(u, torch.float64, p.ndof, "u"),
                             _dev(y, torch.float64, p.ndof, "y")), ctx.handle)
    return y


def to_matvec_f32(ctx: Context, x, u, y=None):
    """x = None reuses the moduli of the previous product on ctx."""
    p = ctx.prob
    if y is None:
        y = torch.empty(p.ndof, dtype=torch.float32, device=u.device)
    _check(L.lib().to_matvec_f32(ctx.handle, _dev(x, torch.float64, p.nel, "x"),
                                 _dev(u, torch.float32, p.ndof, "u"),
                                 _dev(y, torch.float32, p.ndof, "y")), ctx.handle)
    return y


def product_kernel_name(f32=True):
    """Name of the kernel behind to_matvec_f32 (f32) or to_matvec."""
    return "k_matvec<float, 0>" if f32 else "k_matvec<double, 0>"


# The library forms the CG z = D r inside the product (instead of storing z in
# the update) on grids of at least this many nodes, or as TOPO_CG_ZFUSE=0/1
# says; mirrored here to name the kernel a solve launches.
ZFUSE_MIN_NODES = 1 << 19


def cg_zfuse(dims):
    e = os.environ.get("TOPO_CG_ZFUSE")
    if e is not None:
        return int(e) != 0
    return (dims[0] + 1) * (dims[1] + 1) * (dims[2] + 1) >= ZFUSE_MIN_NODES


def cg_product_kernel_name(dims):
    """Name of the float32 inner-CG product kernel of the one-design solve on
    grid `dims` (vector-ALU product)."""
    return "k_cg_matvec1<float, false, false, %d>" % int(cg_zfuse(dims))



class Server:
    """Continuous-batching compliance + sensitivity server (to_server_*).

    submit() copies the densities; the sensitivity lands in a host array kept
    here until the request is returned by poll()."""

    def __init__(self, hbm_budget_bytes, max_slots=64):
        h = ctypes.c_void_p(0)
        st = L.lib().to_server_create(ctypes.c_size_t(int(hbm_budget_bytes)), int(max_slots), None,
                                      ctypes.byref(h))
        if st != L.TO_OK:
            raise TopoError(st, L.lib().to_server_last_error(None).decode())
        self.handle = h
        self._pending = {}

    def _err(self):
        m = L.lib().to_server_last_error(self.handle)
        return m.decode() if m else ""

    def submit(self, prob: Problem, x, tag, want_dc=True):
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        if x.size != prob.nel:
            raise ValueError("x must have nel entries")
        dc = np.empty(prob.nel, dtype=np.float64) if want_dc else None
        cp = prob.to_c()
        st = L.lib().to_server_submit(self.handle, ctypes.byref(cp), ctypes.c_void_p(x.ctypes.data),
                                      None if dc is None else ctypes.c_void_p(dc.ctypes.data),
                                      ctypes.c_uint64(int(tag)))
        if st != L.TO_OK:
            raise TopoError(st, self._err())
        self._pending[int(tag)] = dc
        return st

    def poll(self, cap=1024):
        """List of dicts {tag, c, status, latency_ms, dc} for finished requests."""
        tags = np.zeros(cap, dtype=np.uint64)
        c = np.zeros(cap)
        status = np.zeros(cap, dtype=np.int32)
        lat = np.zeros(cap)
        n = ctypes.c_int32(0)
        st = L.lib().to_server_poll(self.handle, ctypes.c_void_p(tags.ctypes.data),
                                    ctypes.c_void_p(c.ctypes.data), ctypes.c_void_p(status.ctypes.data),
                                    ctypes.c_void_p(lat.ctypes.data), cap, ctypes.byref(n))
        out = []
        for i in range(n.value):
            t = int(tags[i])
            out.append({"tag": t, "c": float(c[i]), "status": int(status[i]),
                        "latency_ms": float(lat[i]), "dc": self._pending.pop(t, None)})
        if st != L.TO_OK and not out:
            raise TopoError(st, self._err())
        return out

    def wait_idle(self, timeout_ms=600000.0):
        return L.lib().to_server_wait_idle(self.handle, float(timeout_ms))

    def stats(self):
        live, queued = ctypes.c_int32(0), ctypes.c_int32(0)
        ticks, free = ctypes.c_int64(0), ctypes.c_size_t(0)
        _check(L.lib().to_server_stats(self.handle, ctypes.byref(live), ctypes.byref(queued),
                                       ctypes.byref(ticks), ctypes.byref(free)))
        return {"live": live.value, "queued": queued.value, "ticks": ticks.value,
                "free_bytes": free.value}

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            L.lib().to_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
